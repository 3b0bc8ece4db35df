// Low-precision distance screens on MFMA and the copies they read: bf16
// (v_mfma_f32_16x16x32_bf16) and OCP fp8 e4m3 with one fp32 scale per vector
// (v_mfma_f32_16x16x32_fp8_fp8).
//
// Same work items and lane layout as the fp32 register screen, with fewer
// bytes per row: lane l holds row (l % 16) and frame (l % 16) and takes the
// 16-byte pieces 4 s + l / 16 of their rows, so the 16 rows of a block are
// read as 64-byte runs. A bf16 piece (8 values) feeds one MFMA, an fp8 piece
// (16 values) two; rows and frames use the same assignment of values to MFMA
// k slots, so every piece of a row meets the same piece of the frame.
// Products are accumulated in fp32 (fp8 products are exact in fp32); the fp8
// sum is multiplied by the frame's and the row's scale. The screen value is
// |q|^2 + |d|^2 - 2 q~.d~ with the norms of the fp32 vectors and the dot
// product of their roundings q~, d~ (for fp8: scale times the e4m3 value);
// its error against the exact distance is bounded by the select kernel from
// |q~ - q| and |q~| (per frame, from the prep kernel) and the largest
// |d~ - d| and |d~| over the rows (from the copy kernels below).
#include "hloc_device.h"
#include "hloc_internal.h"

#include <algorithm>

namespace hloc {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));  // 16-byte piece (native vector)

constexpr float kFp8Max = 448.f;  // largest finite OCP e4m3 value

// Round-to-nearest-even fp32 -> bf16 bits (finite inputs).
__device__ __forceinline__ uint16_t bf16_rne(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Value of an OCP e4m3 byte (sign, 4 exponent bits of bias 7, 3 mantissa
// bits; exponent 0 is subnormal). The two NaN codes are never produced here.
__device__ __forceinline__ float fp8_to_f32(uint32_t b) {
  const int e = (b >> 3) & 15, m = b & 7;
  const float v = e == 0 ? ldexpf((float)m, -9) : ldexpf((float)(8 + m), e - 10);
  return (b & 0x80) ? -v : v;
}

// Nearest e4m3 bytes of x0 and x1 (|x| <= 448), in the low two bytes.
__device__ __forceinline__ uint32_t fp8_pair(float x0, float x1) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x0, x1, 0, false) & 0xFFFFu;
}

__device__ __forceinline__ float clamp_fp8(float x) { return fminf(fmaxf(x, -kFp8Max), kFp8Max); }

constexpr int kLpRowsPerWave = 16;

// Low-precision copy of n rows of dp floats, kLpRowsPerWave rows per wave.
// bf16: dst holds dp 16-bit values per row. fp8: dst holds dp bytes per row
// and scale[i] = max |row| / 448 (1 for a zero row), the row being
// scale[i] * e4m3(row / scale[i]). Per-row FP64 norms of the rounding error
// and of the rounded row; maxima into max_err / max_norm (float bits, one
// atomic per block).
template <int FMT>
__global__ void k_rows_to_lp(const float *__restrict__ src, int64_t n, int dp, void *dst_,
                             float *__restrict__ scale, float *max_err, float *max_norm) {
  __shared__ float s_e[4], s_n[4];
  const int lane = lane_id();
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave_id()) * kLpRowsPerWave;
  float me = 0.f, mn = 0.f;
  for (int64_t i = i0; i < min(n, i0 + kLpRowsPerWave); ++i) {
    const float *r = src + i * dp;
    double e2 = 0.0, n2 = 0.0;
    if (FMT == HLOC_BF16) {
      uint16_t *o = static_cast<uint16_t *>(dst_) + i * dp;
      for (int c = lane; c < dp; c += 64) {
        const uint16_t h = bf16_rne(r[c]);
        o[c] = h;
        const double t = (double)bf16_to_f32(h);
        e2 = fma(t - (double)r[c], t - (double)r[c], e2);
        n2 = fma(t, t, n2);
      }
    } else {
      uint8_t *o = static_cast<uint8_t *>(dst_) + i * dp;
      float amax = 0.f;
      for (int c = lane; c < dp; c += 64) amax = fmaxf(amax, fabsf(r[c]));
      for (int o2 = 32; o2 > 0; o2 >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o2));
      const float sc = amax > 0.f ? amax / kFp8Max : 1.f;
      const float inv = amax > 0.f ? kFp8Max / amax : 1.f;
      if (lane == 0) scale[i] = sc;
      // two values per lane per step: dp is a multiple of 32
      for (int c = 2 * lane; c < dp; c += 128) {
        const uint32_t p = fp8_pair(clamp_fp8(r[c] * inv), clamp_fp8(r[c + 1] * inv));
        o[c] = (uint8_t)p;
        o[c + 1] = (uint8_t)(p >> 8);
        const double t0 = (double)fp8_to_f32(p & 0xFF) * sc, t1 = (double)fp8_to_f32(p >> 8) * sc;
        e2 = fma(t0 - (double)r[c], t0 - (double)r[c], e2);
        e2 = fma(t1 - (double)r[c + 1], t1 - (double)r[c + 1], e2);
        n2 = fma(t0, t0, n2);
        n2 = fma(t1, t1, n2);
      }
    }
    e2 = wave_sum_f64(e2);
    n2 = wave_sum_f64(n2);
    me = fmaxf(me, (float)sqrt(e2));
    mn = fmaxf(mn, (float)sqrt(n2));
  }
  if (lane == 0) {
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

hipError_t launch_rows_to_lp(int32_t fmt, const float *src, int64_t n, int32_t dp, void *dst,
                             float *scale, float *max_err, float *max_norm, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((unsigned)((n + 4 * kLpRowsPerWave - 1) / (4 * kLpRowsPerWave)));
  if (fmt == HLOC_BF16)
    return launch_kernel(k_rows_to_lp<HLOC_BF16>, grid, dim3(256), 0, s, src, n, dp, dst, scale,
                         max_err, max_norm);
  if (fmt == HLOC_FP8)
    return launch_kernel(k_rows_to_lp<HLOC_FP8>, grid, dim3(256), 0, s, src, n, dp, dst, scale,
                         max_err, max_norm);
  return hipErrorInvalidValue;
}

// Per-frame copies for the low-precision screens: the same rounding as the
// rows (fp8: a scale per frame), and the norms of the rounding error (q_err)
// and of the rounded frame (q_lon), rounded up. One wave per frame.
template <int FMT>
__global__ void k_frames_to_lp(const float *__restrict__ qp, int nq, int dp, void *dst_,
                               float *__restrict__ scale, float *__restrict__ q_err,
                               float *__restrict__ q_lon) {
  const int f = blockIdx.x * 4 + wave_id(), lane = lane_id();
  if (f >= nq) return;
  const float *r = qp + (int64_t)f * dp;
  double e2 = 0.0, n2 = 0.0;
  if (FMT == HLOC_BF16) {
    uint16_t *o = static_cast<uint16_t *>(dst_) + (int64_t)f * dp;
    for (int c = lane; c < dp; c += 64) {
      const uint16_t h = bf16_rne(r[c]);
      o[c] = h;
      const double t = (double)bf16_to_f32(h);
      e2 = fma(t - (double)r[c], t - (double)r[c], e2);
      n2 = fma(t, t, n2);
    }
  } else {
    uint8_t *o = static_cast<uint8_t *>(dst_) + (int64_t)f * dp;
    float amax = 0.f;
    for (int c = lane; c < dp; c += 64) amax = fmaxf(amax, fabsf(r[c]));
    for (int o2 = 32; o2 > 0; o2 >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o2));
    const float sc = amax > 0.f ? amax / kFp8Max : 1.f;
    const float inv = amax > 0.f ? kFp8Max / amax : 1.f;
    if (lane == 0) scale[f] = sc;
    for (int c = 2 * lane; c < dp; c += 128) {
      const uint32_t p = fp8_pair(clamp_fp8(r[c] * inv), clamp_fp8(r[c + 1] * inv));
      o[c] = (uint8_t)p;
      o[c + 1] = (uint8_t)(p >> 8);
      const double t0 = (double)fp8_to_f32(p & 0xFF) * sc, t1 = (double)fp8_to_f32(p >> 8) * sc;
      e2 = fma(t0 - (double)r[c], t0 - (double)r[c], e2);
      e2 = fma(t1 - (double)r[c + 1], t1 - (double)r[c + 1], e2);
      n2 = fma(t0, t0, n2);
      n2 = fma(t1, t1, n2);
    }
  }
  e2 = wave_sum_f64(e2);
  n2 = wave_sum_f64(n2);
  if (lane == 0) {
    q_err[f] = (float)sqrt(e2) * (1.0f + 1e-6f);
    q_lon[f] = (float)sqrt(n2) * (1.0f + 1e-6f);
  }
}

hipError_t launch_frames_to_lp(int32_t fmt, const float *qp, int32_t nq, int32_t dp, void *dst,
                               float *scale, float *q_err, float *q_lon, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  const dim3 grid((unsigned)((nq + 3) / 4));
  if (fmt == HLOC_BF16)
    return launch_kernel(k_frames_to_lp<HLOC_BF16>, grid, dim3(256), 0, s, qp, nq, dp, dst, scale,
                         q_err, q_lon);
  if (fmt == HLOC_FP8)
    return launch_kernel(k_frames_to_lp<HLOC_FP8>, grid, dim3(256), 0, s, qp, nq, dp, dst, scale,
                         q_err, q_lon);
  return hipErrorInvalidValue;
}

// One 16-byte piece of a row against the same piece of a frame.
template <int FMT>
__device__ __forceinline__ v4f lp_mfma(uint4 a, uint4 b, v4f acc) {
  if (FMT == HLOC_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), acc, 0, 0, 0);
  } else {
    const long a0 = (long)(((uint64_t)a.y << 32) | a.x), a1 = (long)(((uint64_t)a.w << 32) | a.z);
    const long b0 = (long)(((uint64_t)b.y << 32) | b.x), b1 = (long)(((uint64_t)b.w << 32) | b.z);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
  }
}

// The same on native vectors (kept in registers across loops).
template <int FMT>
__device__ __forceinline__ v4f lp_mfma_v(v4u a, v4u b, v4f acc) {
  if (FMT == HLOC_BF16) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a),
                                                   __builtin_bit_cast(v8bf, b), acc, 0, 0, 0);
  } else {
    const long a0 = (long)(((uint64_t)a.y << 32) | a.x), a1 = (long)(((uint64_t)a.w << 32) | a.z);
    const long b0 = (long)(((uint64_t)b.y << 32) | b.x), b1 = (long)(((uint64_t)b.w << 32) | b.z);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a0, b0, acc, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a1, b1, acc, 0, 0, 0);
  }
}

// Screen word of a row with squared norm rn against a frame with squared norm
// qn, from the low-precision dot product (times the two scales for fp8).
template <int FMT>
__device__ __forceinline__ uint32_t lp_word(float qn, float rn, float acc, float qs, float rs) {
  if (__builtin_isinf(rn)) return 0xFFFFFFFFu;
  const float dot = FMT == HLOC_FP8 ? acc * (qs * rs) : acc;
  float dd = (qn + rn) - 2.f * dot;
  dd = dd > 0.f ? dd : 0.f;
  return __float_as_uint(dd);
}

// Dense items and narrow list items, one item per block, one 16-row block per
// wave, as the fp32 register screen. NS = 16-byte pieces per lane and row
// (row bytes / 64).
template <int FMT, int NS, bool DENSE>
__global__ __launch_bounds__(256) void k_screen_lp(ScreenArgs a) {
  constexpr int ROWU4 = 4 * NS;  // 16-byte pieces per row
  const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const uint4 *rows = static_cast<const uint4 *>(a.rows_lp);
  const uint4 *frames = static_cast<const uint4 *>(a.q_lp);
  int lo = 0, hi, nchunks = 1;
  // dense mode: frames 0 .. nq - 1, or the listed ones
  const int nqd = DENSE && a.frame_list ? *a.frame_count : a.nq;
  if (DENSE) {
    nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    hi = nchunks * ((nqd + kGroup - 1) / kGroup);
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
      gq = min(kGroup, nqd - grp * kGroup);
      fr = grp * kGroup + i;
      if (a.frame_list) fr = i < gq ? a.frame_list[fr] : 0;
      off = (int64_t)fr * a.cap + chunk_row;
    } else {
      row_begin = nx.row_begin;
      chunk_row = nx.chunk_row;
      nrows = nx.nrows_gq >> 16;
      gq = nx.nrows_gq & 0xFFFF;
      if (i < gq) {
        fr = ne.x;
        off = (int64_t)ne.x * a.cap + ne.y + chunk_row / kBlockRows;
      }
      if (itn < hi) nx = a.items[itn];
    }
    if (i >= gq) fr = 0;
    const int nrb = (nrows + 15) >> 4;
    for (int rb = w; rb < nrb; rb += nw) {
      const int rl = min(rb * 16 + i, nrows - 1);
      const uint4 *rp = rows + (int64_t)(row_begin + rl) * ROWU4 + g;
      const uint4 *qp = frames + (int64_t)fr * ROWU4 + g;
      uint4 av[NS], bv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) av[s] = rp[4 * s];
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      const float qn = a.qn2[fr];
      const float qs = FMT == HLOC_FP8 ? a.q_scale[fr] : 1.f;
      v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NS; ++s) acc = lp_mfma<FMT>(av[s], bv[s], acc);
      // the lane's four rows are consecutive rows of its frame's list
      const int row0 = rb * 16 + 4 * g;
      uint32_t wd[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int grow = row_begin + min(row0 + r, nrows - 1);
        const float rs = FMT == HLOC_FP8 ? a.row_scale[grow] : 1.f;
        wd[r] = row0 + r < nrows ? lp_word<FMT>(qn, a.row_n2[grow], acc[r], qs, rs) : 0xFFFFFFFFu;
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

// Wide list items, as the fp32 wide screen: the chunk's rows (and fp8 scales)
// staged in LDS once, a 16-frame group per wave at a time.
template <int FMT, int NS>
__global__ __launch_bounds__(256) void k_screen_wide_lp(ScreenArgs a) {
  constexpr int ROWU4 = 4 * NS;
  constexpr int LDR = ROWU4 + 1;  // pieces per LDS row, one of padding
  extern __shared__ uint4 s_rows[];  // 64 x LDR
  __shared__ float s_rn[64], s_rs[64];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  const int i = lane & 15, g = lane >> 4;
  const uint4 *rows = static_cast<const uint4 *>(a.rows_lp);
  const uint4 *frames = static_cast<const uint4 *>(a.q_lp);
  // the chunk of the block's next item is read into registers (all of a
  // thread's pieces at once) while the current one is screened, with the rq
  // entry of each lane's frame in the wave's first group
  constexpr int PER = 64 * ROWU4 / 256;  // pieces per thread (256 threads)
  static_assert(64 * ROWU4 % 256 == 0, "whole pieces per thread");
  uint4 pv[PER];
  float prn = 0.f, prs = 1.f;
  WideItem wn{};
  int2 pe = make_int2(0, 0);
  auto fetch = [&](int item) {
    wn = wide_item(a, item);
    pe = wide_entry(a, wn, w * kGroup + i);
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * 256, row = e / ROWU4, c = e - row * ROWU4;
      pv[u] = row < wn.nrows ? rows[(int64_t)(wn.row_begin + row) * ROWU4 + c]
                             : make_uint4(0u, 0u, 0u, 0u);
    }
    if (tid < 64) {
      prn = tid < wn.nrows ? a.row_n2[wn.row_begin + tid] : 0.f;
      prs = (FMT == HLOC_FP8 && tid < wn.nrows) ? a.row_scale[wn.row_begin + tid] : 1.f;
    }
  };
  int lo;
  const int hi = wide_range(a, &lo);
  if (lo + (int)blockIdx.x < hi) fetch(lo + blockIdx.x);
  for (int it = lo + blockIdx.x; it < hi; it += gridDim.x) {
    const WideItem wi = wn;
    const int nrows = wi.nrows, gq = wi.gq;
    int2 ce = pe;
    __syncthreads();  // the previous item's rows are no longer read
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * 256, row = e / ROWU4, c = e - row * ROWU4;
      s_rows[row * LDR + c] = pv[u];
    }
    if (tid < 64) {
      s_rn[tid] = prn;
      s_rs[tid] = prs;
    }
    __syncthreads();
    if (it + (int)gridDim.x < hi) fetch(it + gridDim.x);
    for (int grp = w; grp * kGroup < gq; grp += nw) {
      const int gs = min(kGroup, gq - grp * kGroup);
      int fr = 0;
      int64_t off = 0;
      if (i < gs) wide_frame(a, wi, grp * kGroup + i, ce, &fr, &off);
      const uint4 *qp = frames + (int64_t)fr * ROWU4 + g;
      uint4 bv[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) bv[s] = qp[4 * s];
      const float qn = a.qn2[fr];
      const float qs = FMT == HLOC_FP8 ? a.q_scale[fr] : 1.f;
      ce = wide_entry(a, wi, (grp + nw) * kGroup + i);  // the wave's next group
      uint32_t bm[4];  // list items: the frame's block words of the chunk
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        bm[rb] = 0xFFFFFFFFu;
        if (rb * 16 >= nrows) continue;
        const uint4 *rp = s_rows + (rb * 16 + i) * LDR + g;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < NS; ++s) acc = lp_mfma<FMT>(rp[4 * s], bv[s], acc);
        // the lane's four rows are consecutive rows of its frame's list
        const int row0 = rb * 16 + 4 * g;
        uint32_t wd[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(row0 + r, 63);
          wd[r] = row0 + r < nrows ? lp_word<FMT>(qn, s_rn[row], acc[r], qs, s_rs[row])
                                   : 0xFFFFFFFFu;
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

// Wide list items with the rows held in registers and the frames staged
// through LDS, 16 at a time, double-buffered (wide items of the bf16 and fp8
// screens when the padded length gives NS % 4 == 0).
// A block of four waves takes one wide item: up to kWideRunsRs runs of 128
// rows of one region against the item's gq frames. For each run, wave w
// holds rows 32 w .. 32 w + 31 as the MFMA A operand (two 16-row tiles over
// the whole padded length), so each row is read from memory once per item
// and every LDS read of a frame piece feeds both row tiles (two MFMAs for
// bf16, four for fp8). The item's frame entries are staged in LDS once; its
// frame groups then stream through the two buffers run after run: while one
// (run, group) step is multiplied, the next step's group is read into
// registers (across a run boundary that is group 0 again) and written to the
// other buffer after the multiply. The last step of a run requests the next
// run's rows as soon as its multiply has read the current ones; it is
// written apart from the run's other steps so that no other step has row
// loads in flight, and the multiply of a step never waits for the next
// step's frame group. An item's set-up requests its entries, then its first
// frame group, its first run and the entries' norms together; the next
// item's descriptor is requested one item ahead.
// The epilogue takes, per frame and row tile, the smallest of the tile's 16
// screen words (the block word) and stores it at the frame's block position.
// Items are dealt to the XCDs in contiguous runs (blocks go to the eight
// XCDs round-robin): the chunks of one region, which stage the same frames,
// run on one XCD and find them in its L2.
constexpr int kRsAhead = 4;  // frame pieces in flight ahead of the multiplies

template <int FMT, int NS>
__global__ __launch_bounds__(256) void k_screen_wide_rs(ScreenArgs a) {
  constexpr int ROWU4 = 4 * NS;                 // 16-byte pieces per row
  constexpr int LDF = ROWU4 + 1;                // padded frame row in LDS
  constexpr int TPF = 256 / kGroup;             // threads staging one frame
  static_assert(ROWU4 % TPF == 0, "whole pieces per thread");
  constexpr int PERF = ROWU4 / TPF;             // pieces per thread per group
  constexpr int U = kListFrames / 256;          // item entries per thread
  extern __shared__ v4u s_fr[];                 // 2 x kGroup x LDF
  // the item's frames: rq entries, squared norms, scales (read once per item)
  __shared__ int2 s_e[kListFrames];
  __shared__ float s_qn[kListFrames], s_qs[kListFrames];
  const int tid = threadIdx.x, lane = lane_id(), w = wave_id();
  const int i = lane & 15, g = lane >> 4;
  const v4u *rows = static_cast<const v4u *>(a.rows_lp);
  const v4u *frames = static_cast<const v4u *>(a.q_lp);
  int lo;
  const int hi = wide_range(a, &lo);
  // this block's run of items: XCD x = b % 8 owns [x span, (x + 1) span)
  constexpr int kXcd = 8;
  const int nb = gridDim.x / kXcd, x = blockIdx.x % kXcd, jb = blockIdx.x / kXcd;
  const int span = (hi - lo + kXcd - 1) / kXcd;
  const int it0 = lo + x * span, it1 = min(hi, it0 + span);
  // staging: thread t loads pieces (t % TPF) + TPF u of frame t / TPF
  const int sj = tid / TPF, sc = tid % TPF;
  // With item counters the blocks of XCD x take the items of x's span in
  // order, one counter increment each, then those left in the other spans
  // (x + 1, x + 2, ... mod 8), so no block idles while items remain; thread
  // 0 takes the next item at an item's start and the block reads it after
  // the item's first barrier (two slots by item parity: the slot thread 0
  // writes was last read before the previous item's set-up barrier). Without
  // them block jb of XCD x takes items it0 + jb, + nb, ...
  const bool dyn = a.item_ctr != nullptr;
  __shared__ int s_nx[2];
  int xs = 0;  // spans thread 0 has emptied
  auto grab = [&]() -> int {
    while (xs < kXcd) {
      const int xx = x + xs < kXcd ? x + xs : x + xs - kXcd;
      const int b0 = lo + xx * span, b1 = min(hi, b0 + span);
      const int j = atomicAdd(a.item_ctr + xx, 1);
      if (b0 + j < b1) return b0 + j;
      ++xs;
    }
    return hi;
  };
  int it = it0 + jb, lim = it1;
  if (dyn) {
    if (tid == 0) s_nx[0] = grab();
    __syncthreads();
    it = s_nx[0];
    lim = hi;
  }
  Item nxt = it < lim ? a.items[it] : Item{};
  for (int par = 1; it < lim; par ^= 1) {
    const Item cur = nxt;
    int itn = it + nb;
    if (dyn) {
      if (tid == 0) s_nx[par] = grab();
    } else if (itn < lim) {
      nxt = a.items[itn];
    }
    const int row_begin = cur.row_begin, chunk_row = cur.chunk_row, q0 = cur.q0;
    const int nrows = cur.nrows_gq >> 16, gq = cur.nrows_gq & 0xFFFF;
    const int nrun = (nrows + kWideRowsRs - 1) / kWideRowsRs;
    const int ng = (gq + kGroup - 1) / kGroup;
    const int nst = nrun * ng;  // (run, group) steps, groups inner
    v4u av[2][NS];
    float rn[2][4], rs[2][4];
    v4u pv[PERF];
    // the wave's rows of run C (clamped to the item's last row; words of rows
    // past it are no candidates), then their norms and scales
#define HLOC_RS_ROWS(C)                                                          \
  _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                \
    const int rl = min((C) * kWideRowsRs + 32 * w + 16 * h + i, nrows - 1);      \
    const v4u *rp = rows + (int64_t)(row_begin + rl) * ROWU4 + g;                \
    _Pragma("unroll") for (int s = 0; s < NS; ++s) av[h][s] = rp[4 * s];         \
  }
#define HLOC_RS_NORMS(C)                                                         \
  _Pragma("unroll") for (int h = 0; h < 2; ++h) {                                \
    _Pragma("unroll") for (int r = 0; r < 4; ++r) {                              \
      const int row = (C) * kWideRowsRs + 32 * w + 16 * h + 4 * g + r;           \
      const int grow = row_begin + min(row, nrows - 1);                          \
      rn[h][r] = row < nrows ? a.row_n2[grow] : __builtin_inff();                \
      rs[h][r] = FMT == HLOC_FP8 ? a.row_scale[grow] : 1.f;                      \
    }                                                                            \
  }
#define HLOC_RS_FETCH_FRAME(FR)                                                  \
  {                                                                              \
    const v4u *fp = frames + (int64_t)(FR) * ROWU4 + sc;                         \
    _Pragma("unroll") for (int u = 0; u < PERF; ++u) pv[u] = fp[TPF * u];        \
  }
#define HLOC_RS_STAGE(BUF)                                                       \
  {                                                                              \
    _Pragma("unroll") for (int u = 0; u < PERF; ++u)                             \
        s_fr[((BUF) * kGroup + sj) * LDF + sc + TPF * u] = pv[u];                \
  }
    __syncthreads();  // the previous item's entries and frames are no longer read
    if (dyn) {
      itn = s_nx[par];
      if (itn < lim) nxt = a.items[itn];
    }
    {
      // the item's frame entries (frames past gq: frame 0, never stored) and
      // the frame of this thread's piece of the first group
      const int2 ef = sj < gq ? a.rq[q0 + sj] : make_int2(0, 0);
      int2 e[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = u * 256 + tid;
        e[u] = j < gq ? a.rq[q0 + j] : make_int2(0, 0);
      }
      // the first group, the first run and the entries' norms together
      HLOC_RS_FETCH_FRAME(ef.x)
      float qv[U], sv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        qv[u] = a.qn2[e[u].x];
        sv[u] = FMT == HLOC_FP8 ? a.q_scale[e[u].x] : 1.f;
      }
      HLOC_RS_ROWS(0)
      HLOC_RS_NORMS(0)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = u * 256 + tid;
        if (j < ng * kGroup) {
          s_e[j] = e[u];
          s_qn[j] = qv[u];
          s_qs[j] = sv[u];
        }
      }
      HLOC_RS_STAGE(0)
    }
    __syncthreads();
    // one (run c, group K) step; LAST: the run's last group
#define HLOC_RS_STEP(K, LAST)                                                    \
  {                                                                              \
    const int buf = st & 1;                                                      \
    const bool more = st + 1 < nst;                                              \
    if (more) HLOC_RS_FETCH_FRAME(s_e[((LAST) ? 0 : (K) + 1) * kGroup + sj].x)   \
    v4f acc[2] = {v4f{0.f, 0.f, 0.f, 0.f}, v4f{0.f, 0.f, 0.f, 0.f}};             \
    const v4u *bp = s_fr + (buf * kGroup + i) * LDF + g;                         \
    /* frame pieces read kRsAhead steps ahead of their multiplies, the */       \
    /* order pinned: the first reads, then per k step two multiplies and */     \
    /* the next read */                                                          \
    v4u bq[NS];                                                                  \
    _Pragma("unroll") for (int s = 0; s < kRsAhead && s < NS; ++s) bq[s] = bp[4 * s]; \
    __builtin_amdgcn_sched_group_barrier(0x100, kRsAhead < NS ? kRsAhead : NS, 0); \
    _Pragma("unroll") for (int s = 0; s < NS; ++s) {                             \
      if (s + kRsAhead < NS) bq[s + kRsAhead] = bp[4 * (s + kRsAhead)];          \
      acc[0] = lp_mfma_v<FMT>(av[0][s], bq[s], acc[0]);                          \
      acc[1] = lp_mfma_v<FMT>(av[1][s], bq[s], acc[1]);                          \
      __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);                         \
      if (s + kRsAhead < NS) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  \
    }                                                                            \
    if ((LAST) && more) HLOC_RS_ROWS(c + 1)                                      \
    const int2 e = s_e[(K) * kGroup + i];                                        \
    const float qn = s_qn[(K) * kGroup + i], qs = s_qs[(K) * kGroup + i];        \
    const bool fok = (K) * kGroup + i < gq;                                      \
    const int blk = (chunk_row + c * kWideRowsRs) / kBlockRows;                  \
    _Pragma("unroll") for (int h = 0; h < 2; ++h) {                              \
      if (c * kWideRowsRs + 32 * w + 16 * h < nrows) { /* (uniform) */           \
        uint32_t wd[4];                                                          \
        _Pragma("unroll") for (int r = 0; r < 4; ++r)                            \
            wd[r] = lp_word<FMT>(qn, rn[h][r], acc[h][r], qs, rs[h][r]);         \
        const uint32_t m = block_min16(wd);                                      \
        if (fok && g == 0) a.cand[(int64_t)e.x * a.cap + e.y + blk + 2 * w + h] = m; \
      }                                                                          \
    }                                                                            \
    if ((LAST) && more) HLOC_RS_NORMS(c + 1)                                     \
    if (more) HLOC_RS_STAGE(buf ^ 1)                                             \
    __syncthreads();                                                             \
    ++st;                                                                        \
  }
    int st = 0;  // steps done
    for (int c = 0; c < nrun; ++c) {
      for (int k = 0; k + 1 < ng; ++k) HLOC_RS_STEP(k, false)
      HLOC_RS_STEP(ng - 1, true)
    }
#undef HLOC_RS_STEP
#undef HLOC_RS_ROWS
#undef HLOC_RS_NORMS
#undef HLOC_RS_FETCH_FRAME
#undef HLOC_RS_STAGE
    it = itn;
  }
}

template <int NS>
size_t wide_lp_lds_bytes() {
  return (size_t)64 * (4 * NS + 1) * sizeof(uint4);
}

template <int NS>
constexpr size_t wide_rs_lds_bytes() {
  return (size_t)2 * kGroup * (4 * NS + 1) * sizeof(v4u);
}
constexpr int kRsBlocksPerCu = 2;  // blocks per compute unit if the occupancy query fails

// Pieces per lane for a padded length: bf16 rows take dp / 32, fp8 rows
// dp / 64 (0: no kernel for this length).
int lp_pieces(int32_t fmt, int32_t dp) {
  const int bytes = fmt == HLOC_BF16 ? 2 * dp : fmt == HLOC_FP8 ? dp : 0;
  if (bytes <= 0 || bytes % 64 != 0) return 0;
  switch (bytes / 64) {
    case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 12: case 16:
      return bytes / 64;
    default:
      return 0;
  }
}

bool lp_screen_supports(int32_t fmt, int32_t dp) { return lp_pieces(fmt, dp) > 0; }

bool lp_wide_rs(int32_t fmt, int32_t dp) {
  const int ns = lp_pieces(fmt, dp);
  return ns > 0 && ns % 4 == 0;
}

template <int FMT, int NS>
hipError_t launch_lp_ns(const ScreenArgs &a, int32_t grid, int32_t wide_cu, hipStream_t s) {
  if constexpr (NS % 4 == 0) {
    if (wide_cu > 0 && !a.dense) {
      // as many blocks as the compute units hold at once (registers and LDS)
      static int per_cu = 0;
      if (per_cu == 0) {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &occ, reinterpret_cast<const void *>(&k_screen_wide_rs<FMT, NS>), 256,
                wide_rs_lds_bytes<NS>()) != hipSuccess || occ < 1) {
          (void)hipGetLastError();
          occ = kRsBlocksPerCu;
        }
        per_cu = occ;
      }
      // every block resident at once, a multiple of the eight XCDs
      const int64_t resident = std::max<int64_t>(8, (int64_t)wide_cu * per_cu / 8 * 8);
      return launch_kernel(k_screen_wide_rs<FMT, NS>, dim3((int32_t)resident), dim3(256),
                           (uint32_t)wide_rs_lds_bytes<NS>(), s, a);
    }
  }
  if (wide_cu > 0) {
    const int64_t resident =
        (int64_t)wide_cu * std::max<int64_t>(1, kLdsPerCu / wide_lp_lds_bytes<NS>());
    return launch_kernel(k_screen_wide_lp<FMT, NS>, dim3((int32_t)std::min<int64_t>(grid, resident)),
                         dim3(256), (uint32_t)wide_lp_lds_bytes<NS>(), s, a);
  }
  return a.dense ? launch_kernel(k_screen_lp<FMT, NS, true>, dim3(grid), dim3(256), 0, s, a)
                 : launch_kernel(k_screen_lp<FMT, NS, false>, dim3(grid), dim3(256), 0, s, a);
}

// wide_cu: compute units for the wide kernel, 0 for the narrow one
template <int FMT>
hipError_t launch_lp_fmt(const ScreenArgs &a, int32_t grid, int32_t wide_cu, hipStream_t s) {
  switch (lp_pieces(FMT, a.dp)) {
#define HLOC_LP_CASE(N) \
  case N:               \
    return launch_lp_ns<FMT, N>(a, grid, wide_cu, s);
    HLOC_LP_CASE(1)
    HLOC_LP_CASE(2)
    HLOC_LP_CASE(3)
    HLOC_LP_CASE(4)
    HLOC_LP_CASE(5)
    HLOC_LP_CASE(6)
    HLOC_LP_CASE(8)
    HLOC_LP_CASE(10)
    HLOC_LP_CASE(12)
    HLOC_LP_CASE(16)
#undef HLOC_LP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_screen_lp(int32_t fmt, const ScreenArgs &a, int32_t grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  if (a.rows_per_item % 16 != 0) return hipErrorInvalidValue;
  if (fmt == HLOC_BF16) return launch_lp_fmt<HLOC_BF16>(a, grid, 0, s);
  if (fmt == HLOC_FP8) return launch_lp_fmt<HLOC_FP8>(a, grid, 0, s);
  return hipErrorInvalidValue;
}

hipError_t launch_screen_wide_lp(int32_t fmt, const ScreenArgs &a, int32_t grid, int32_t num_cu,
                                 hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  num_cu = std::max(num_cu, 1);
  if (a.rows_per_item % 16 != 0 || (a.dense && a.rows_per_item > kWideRows))
    return hipErrorInvalidValue;
  if (fmt == HLOC_BF16) return launch_lp_fmt<HLOC_BF16>(a, grid, num_cu, s);
  if (fmt == HLOC_FP8) return launch_lp_fmt<HLOC_FP8>(a, grid, num_cu, s);
  return hipErrorInvalidValue;
}

// LDS limits of the wide kernels (above the 64 KB default).
hipError_t prepare_screen_lp_kernels() {
#define HLOC_LP_ATTR(F, N)                                                                 \
  {                                                                                        \
    const hipError_t e = hipFuncSetAttribute(                                              \
        reinterpret_cast<const void *>(&k_screen_wide_lp<F, N>),                           \
        hipFuncAttributeMaxDynamicSharedMemorySize, (int)wide_lp_lds_bytes<N>());          \
    if (e != hipSuccess) return e;                                                         \
  }
#define HLOC_LP_ATTRS(F) \
  HLOC_LP_ATTR(F, 1)     \
  HLOC_LP_ATTR(F, 2)     \
  HLOC_LP_ATTR(F, 3)     \
  HLOC_LP_ATTR(F, 4)     \
  HLOC_LP_ATTR(F, 5)     \
  HLOC_LP_ATTR(F, 6)     \
  HLOC_LP_ATTR(F, 8)     \
  HLOC_LP_ATTR(F, 10)    \
  HLOC_LP_ATTR(F, 12)    \
  HLOC_LP_ATTR(F, 16)
  HLOC_LP_ATTRS(HLOC_BF16)
  HLOC_LP_ATTRS(HLOC_FP8)
#undef HLOC_LP_ATTRS
#undef HLOC_LP_ATTR
  return hipSuccess;
}

}  // namespace hloc
