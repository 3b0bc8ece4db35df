// BF16 distance screen on MFMA (gfx950 v_mfma_f32_16x16x32_bf16) and the
// bf16 copies it reads.
//
// Same work items and lane layout as the fp32 register screen, with half the
// bytes per row: for each 32-wide k block lane l holds row (l % 16) and
// frame (l % 16)'s eight bf16 values at k = 32 s + 8 (l / 16) .. + 7, so one
// 16-byte load feeds one MFMA and the 16 rows of a block are read as 64-byte
// runs. Products are accumulated in fp32. The screen value is
// |q|^2 + |d|^2 - 2 q~.d~ with the norms of the fp32 vectors and the dot
// product of their bf16 roundings q~, d~; its error against the exact
// distance is bounded by the select kernel from |q~ - q| (per frame) and the
// largest |d~ - d| and |d~| over the database (see the design notes).
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// Round-to-nearest-even fp32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr int kBf16RowsPerWave = 16;

// bf16 copy of n rows, kBf16RowsPerWave rows per wave; per-row FP64 norms of
// the rounding error and of the rounded row, maxima into max_err / max_norm
// (float bits, one atomic per block).
__global__ void k_rows_to_bf16(const float *__restrict__ src, int64_t n, int dp,
                               uint16_t *__restrict__ dst, float *max_err, float *max_norm) {
  __shared__ float s_e[4], s_n[4];
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave_id()) * kBf16RowsPerWave;
  float me = 0.f, mn = 0.f;
  for (int64_t i = i0; i < min(n, i0 + kBf16RowsPerWave); ++i) {
    const float *r = src + i * dp;
    uint16_t *o = dst + i * dp;
    double e2 = 0.0, n2 = 0.0;
    for (int c = lane_id(); c < dp; c += 64) {
      const uint16_t h = bf16_rne(r[c]);
      o[c] = h;
      const double t = (double)bf16_to_f32(h);
      e2 = fma(t - (double)r[c], t - (double)r[c], e2);
      n2 = fma(t, t, n2);
    }
    e2 = wave_sum_f64(e2);
    n2 = wave_sum_f64(n2);
    me = fmaxf(me, (float)sqrt(e2));
    mn = fmaxf(mn, (float)sqrt(n2));
  }
  if (lane_id() == 0) {
    s_e[wave_id()] = me;
    s_n[wave_id()] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w) {
      s_e[0] = fmaxf(s_e[0], s_e[w]);
      s_n[0] = fmaxf(s_n[0], s_n[w]);
    }
    atomicMax(reinterpret_cast<unsigned int *>(max_err), __float_as_uint(s_e[0]));
    atomicMax(reinterpret_cast<unsigned int *>(max_norm), __float_as_uint(s_n[0]));
  }
}

hipError_t launch_rows_to_bf16(const float *src, int64_t n, int32_t dp, uint16_t *dst,
                               float *max_err, float *max_norm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t per_block = 4 * kBf16RowsPerWave;
  return launch_kernel(k_rows_to_bf16, dim3((unsigned)((n + per_block - 1) / per_block)),
                       dim3(256), 0, s, src, n, dp, dst, max_err, max_norm);
}

// Dense items and narrow list items, one item per block, one 16-row block per
// wave, as the fp32 register screen.
template <int NS, bool DENSE>  // NS = dp / 32
__global__ __launch_bounds__(256) void k_screen_bf16(ScreenArgs a) {
  constexpr int DP = NS * 32;
  const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  int lo = 0, hi, nchunks = 1;
  if (DENSE) {
    nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    hi = nchunks * ((a.nq + kGroup - 1) / kGroup);
  } else {
    hi = a.n_items[4];  // the narrow items: at most kGroup frames each
  }
  for (int it = lo + blockIdx.x; it < hi; it += gridDim.x) {
    int row_begin, chunk_row, nrows, gq, fr = 0;
    int64_t off = 0;
    if (DENSE) {
      const int c = it % nchunks, grp = it / nchunks;
      row_begin = c * a.rows_per_item;
      chunk_row = row_begin;
      nrows = min(a.rows_per_item, a.nrows - row_begin);
      gq = min(kGroup, a.nq - grp * kGroup);
      fr = grp * kGroup + i;
      off = (int64_t)fr * a.cap + chunk_row;
    } else {
      const Item itm = a.items[it];
      row_begin = itm.row_begin;
      chunk_row = itm.chunk_row;
      nrows = itm.nrows_gq >> 16;
      gq = itm.nrows_gq & 0xFFFF;
      if (i < gq) {
        const int2 e = a.rq[itm.q0 + i];
        fr = e.x;
        off = (int64_t)e.x * a.cap + e.y + chunk_row;
      }
    }
    if (i >= gq) fr = 0;
    const int nrb = (nrows + 15) >> 4;
    for (int rb = w; rb < nrb; rb += nw) {
      const int rl = min(rb * 16 + i, nrows - 1);
      const uint4 *rp = reinterpret_cast<const uint4 *>(a.rows16 + (int64_t)(row_begin + rl) * DP) + g;
      const uint4 *qp = reinterpret_cast<const uint4 *>(a.qp16 + (int64_t)fr * DP) + g;
      uint4 av[NS], bv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) av[s] = rp[4 * s];
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      const float qn = a.qn2[fr];
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av[s]),
                                                      __builtin_bit_cast(v8bf, bv[s]), acc, 0,
                                                      0, 0);
      if (i < gq) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb * 16 + 4 * g + r;
          if (row < nrows) {
            const int grow = row_begin + row;
            const float rn = a.row_n2[grow];
            uint32_t word = 0xFFFFFFFFu;
            if (!__builtin_isinf(rn)) {
              float dd = (qn + rn) - 2.f * acc[r];
              dd = dd > 0.f ? dd : 0.f;
              word = __float_as_uint(dd);
            }
            a.cand[off + row] = word;
          }
        }
      }
    }
  }
}

// Wide list items, as the fp32 wide screen: the chunk's bf16 rows staged in
// LDS once, a 16-frame group per wave at a time.
template <int NS>  // NS = dp / 32
__global__ __launch_bounds__(256) void k_screen_wide_bf16(ScreenArgs a) {
  constexpr int DP = NS * 32;
  constexpr int LDR = 4 * NS + 1;  // uint4 per LDS row, one of padding
  extern __shared__ uint4 s_rows16[];  // 64 x LDR
  __shared__ float s_rn[64];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const int lo = a.n_items[4], hi = a.n_items[0];
  for (int it = lo + blockIdx.x; it < hi; it += gridDim.x) {
    const Item itm = a.items[it];
    const int row_begin = itm.row_begin, chunk_row = itm.chunk_row;
    const int nrows = itm.nrows_gq >> 16, gq = itm.nrows_gq & 0xFFFF;
    __syncthreads();  // the previous item's rows are no longer read
    for (int e = tid; e < 64 * 4 * NS; e += blockDim.x) {
      const int row = e / (4 * NS), c = e - row * (4 * NS);
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (row < nrows) v = reinterpret_cast<const uint4 *>(a.rows16 + (int64_t)(row_begin + row) * DP)[c];
      s_rows16[row * LDR + c] = v;
    }
    if (tid < 64) s_rn[tid] = tid < nrows ? a.row_n2[row_begin + tid] : 0.f;
    __syncthreads();
    for (int grp = w; grp * kGroup < gq; grp += nw) {
      const int gs = min(kGroup, gq - grp * kGroup);
      int fr = 0;
      int64_t off = 0;
      if (i < gs) {
        const int2 e = a.rq[itm.q0 + grp * kGroup + i];
        fr = e.x;
        off = (int64_t)e.x * a.cap + e.y + chunk_row;
      }
      const uint4 *qp = reinterpret_cast<const uint4 *>(a.qp16 + (int64_t)fr * DP) + g;
      uint4 bv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      const float qn = a.qn2[fr];
      for (int rb = 0; rb * 16 < nrows; ++rb) {
        const uint4 *rp = s_rows16 + (rb * 16 + i) * LDR + g;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s)
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, rp[4 * s]),
                                                        __builtin_bit_cast(v8bf, bv[s]), acc, 0,
                                                        0, 0);
        if (i < gs) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rb * 16 + 4 * g + r;
            if (row < nrows) {
              const float rn = s_rn[row];
              uint32_t word = 0xFFFFFFFFu;
              if (!__builtin_isinf(rn)) {
                float dd = (qn + rn) - 2.f * acc[r];
                dd = dd > 0.f ? dd : 0.f;
                word = __float_as_uint(dd);
              }
              a.cand[off + row] = word;
            }
          }
        }
      }
    }
  }
}

template <int NS>
size_t wide16_lds_bytes() {
  return (size_t)64 * (4 * NS + 1) * sizeof(uint4);
}

template <int NS, bool DENSE>
hipError_t launch_bf16_t(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  return launch_kernel(k_screen_bf16<NS, DENSE>, dim3(grid), dim3(256), 0, s, a);
}

hipError_t launch_screen_bf16(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (a.rows_per_item % 16 != 0) return hipErrorInvalidValue;
  switch (a.dp) {
#define HLOC_BF16_CASE(DPV)                                     \
  case DPV:                                                    \
    return a.dense ? launch_bf16_t<DPV / 32, true>(a, grid, s) \
                   : launch_bf16_t<DPV / 32, false>(a, grid, s);
    HLOC_BF16_CASE(32)
    HLOC_BF16_CASE(64)
    HLOC_BF16_CASE(96)
    HLOC_BF16_CASE(128)
    HLOC_BF16_CASE(160)
    HLOC_BF16_CASE(192)
    HLOC_BF16_CASE(256)
    HLOC_BF16_CASE(320)
    HLOC_BF16_CASE(384)
    HLOC_BF16_CASE(512)
#undef HLOC_BF16_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_screen_wide_bf16(const ScreenArgs &a, int32_t grid, hipStream_t s) {
  if (grid <= 0 || a.dense) return hipSuccess;
  if (a.rows_per_item % 16 != 0 || a.rows_per_item > 64) return hipErrorInvalidValue;
  switch (a.dp) {
#define HLOC_BF16_WIDE_CASE(DPV)                                                         \
  case DPV:                                                                              \
    return launch_kernel(k_screen_wide_bf16<DPV / 32>, dim3(grid), dim3(256),              \
                         (uint32_t)wide16_lds_bytes<DPV / 32>(), s, a);
    HLOC_BF16_WIDE_CASE(32)
    HLOC_BF16_WIDE_CASE(64)
    HLOC_BF16_WIDE_CASE(96)
    HLOC_BF16_WIDE_CASE(128)
    HLOC_BF16_WIDE_CASE(160)
    HLOC_BF16_WIDE_CASE(192)
    HLOC_BF16_WIDE_CASE(256)
    HLOC_BF16_WIDE_CASE(320)
    HLOC_BF16_WIDE_CASE(384)
    HLOC_BF16_WIDE_CASE(512)
#undef HLOC_BF16_WIDE_CASE
    default:
      return hipErrorInvalidValue;
  }
}

// LDS limits of the wide bf16 kernels (above the 64 KB default).
hipError_t prepare_screen_bf16_kernels() {
#define HLOC_BF16_WIDE_ATTR(DPV)                                                          \
  {                                                                                       \
    const hipError_t e = hipFuncSetAttribute(                                             \
        reinterpret_cast<const void *>(&k_screen_wide_bf16<DPV / 32>),                     \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)wide16_lds_bytes<DPV / 32>());    \
    if (e != hipSuccess) return e;                                                        \
  }
  HLOC_BF16_WIDE_ATTR(32)
  HLOC_BF16_WIDE_ATTR(64)
  HLOC_BF16_WIDE_ATTR(96)
  HLOC_BF16_WIDE_ATTR(128)
  HLOC_BF16_WIDE_ATTR(160)
  HLOC_BF16_WIDE_ATTR(192)
  HLOC_BF16_WIDE_ATTR(256)
  HLOC_BF16_WIDE_ATTR(320)
  HLOC_BF16_WIDE_ATTR(384)
  HLOC_BF16_WIDE_ATTR(512)
#undef HLOC_BF16_WIDE_ATTR
  return hipSuccess;
}

bool bf16_screen_supports(int32_t dp) {
  switch (dp) {
    case 32: case 64: case 96: case 128: case 160: case 192: case 256: case 320: case 384:
    case 512:
      return true;
    default:
      return false;
  }
}

}  // namespace hloc
