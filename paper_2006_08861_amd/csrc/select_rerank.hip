// Top candidates per frame ("select top candidates", Algorithm 1), one block
// per frame, in one kernel:
//   1. select: the L + 1 smallest (screen word, position) pairs, the word
//      being the float bits of the screen distance (the bits of a
//      non-negative float order like its value). The words are cached in
//      LDS; one histogram of the kDigitBits leading bits below the prefix
//      shared by the smallest and the largest word finds the bucket of the
//      (L+1)-th, and the words of that bucket and of all below it (usually a
//      few more than L + 1) are collected and sorted. If they are too many, a
//      radix select over kDigitBits per pass finds the (L+1)-th word and the
//      survivors are gathered in position order;
//   2. rerank: the positions of the L smallest (the survivors) are mapped to
//      source rows through the frame's region slots (a position is a row, or
//      in the fine stage a 16-row block whose word is the smallest of its
//      rows' screen words, and then each of its rows), then FP64 direct sum
//      of (q_i - d_i)^2, ordered by (distance, tie id) with tie id = original
//      row index (fine stage) or region id (coarse stage);
//   3. certificate: the (L+1)-th word is the best rejected screen distance; if
//      it minus the screen's error bound does not exceed the m-th reranked
//      distance, the block also re-scores every rejected candidate within that
//      bound (in chunks merged with the best m if there are many) and counts
//      the frame.
// Distances are squared L2 (same order as the Euclidean distance of Section 4).
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

constexpr int kWordCache = 27648;  // screen words of a frame kept in (dynamic) LDS
constexpr int kBigFrame = 4096;    // candidate capacity above which a frame gets 1024 threads
constexpr int kMaxSlots = 1024;    // region slots of a frame kept in (dynamic) LDS
constexpr uint32_t kWordNone = 0xFFFFFFFFu;  // no candidate at this position
constexpr uint32_t kNoRow = 0xFFFFFFFFu;     // a block's row slot past its last row
constexpr int kDigitBits = 12;     // radix digit of the select (two passes cover 24 bits)

// Wave reductions: the exchanges 32 and 16 lanes apart through the lane
// swaps (VALU), the rest through shuffles.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  v = min(v, lane_xor32(v));
  v = min(v, lane_xor16(v));
  for (int o = 8; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, lane_xor32(v));
  v = max(v, lane_xor16(v));
  for (int o = 8; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
  v += (int)lane_xor32((uint32_t)v);
  v += (int)lane_xor16((uint32_t)v);
  for (int o = 8; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t y;
    if (o >= 16) {
      const uint32_t lo = o == 32 ? lane_xor32((uint32_t)v) : lane_xor16((uint32_t)v);
      const uint32_t hi = o == 32 ? lane_xor32((uint32_t)(v >> 32)) : lane_xor16((uint32_t)(v >> 32));
      y = ((uint64_t)hi << 32) | lo;
    } else {
      y = (uint64_t)__shfl_xor((long long)v, o);
    }
    v = y < v ? y : v;
  }
  return v;
}

struct SelShared {
  uint32_t sel[kMaxSurvivors + 1];  // candidate positions of the survivors (+ band)
  uint32_t srow[kMaxSurvivors];     // their source rows
  uint64_t sort_hi[kMaxSurvivors];
  uint32_t sort_lo[kMaxSurvivors];
  alignas(16) int hist[1 << kDigitBits];
  int red_i[16];
  int red_j[16];
  uint32_t red_u[16];
  uint32_t red_v[16];
  uint64_t red_k[16];
  uint32_t word;
  int krem;
  int eq;
  int flag;
};

// Inclusive scan over the block of one int per thread (blockDim.x <= 1024):
// a shuffle scan inside each wave, then the wave totals. Two barriers.
__device__ __forceinline__ int block_incl_scan(int v, int *wave_tot) {
  const int lane = lane_id(), w = wave_id(), nw = blockDim.x >> 6;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o);
    if (lane >= o) v += y;
  }
  if (lane == 63) wave_tot[w] = v;
  __syncthreads();
  for (int i = 0; i < w; ++i) v += wave_tot[i];
  (void)nw;
  return v;
}

// The same for two ints per thread at once.
__device__ __forceinline__ void block_incl_scan2(int &v, int &u, int *tot_v, int *tot_u) {
  const int lane = lane_id(), w = wave_id();
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o), z = __shfl_up(u, o);
    if (lane >= o) {
      v += y;
      u += z;
    }
  }
  if (lane == 63) {
    tot_v[w] = v;
    tot_u[w] = u;
  }
  __syncthreads();
  for (int i = 0; i < w; ++i) {
    v += tot_v[i];
    u += tot_u[i];
  }
}

// Block-wide radix select over 32-bit words: returns the target-th smallest
// (1-based) of get(i), i < n, ignoring 0xFFFFFFFF (no candidate); every other
// word lies in [lo, hi]. *krem_out receives its rank among equal words and
// *eq_out how many words equal it. Leading bits shared by lo and hi are
// skipped; the rest are resolved kDigitBits per pass with an LDS histogram.
template <class Get>
__device__ uint32_t block_select_u32(Get get, int n, uint32_t lo, uint32_t hi, int target,
                                     SelShared &sh, int *krem_out, int *eq_out) {
  const int tid = threadIdx.x;
  const uint32_t diff = lo ^ hi;
  const int done = diff ? __clz(diff) : 32;
  uint32_t prefix = done == 32 ? lo : (done ? lo >> (32 - done) : 0u);
  int krem = target, eq = 0;
  int remaining = 32 - done;
  if (remaining == 0) {
    // every word equals lo
    int c = 0;
    for (int i = tid; i < n; i += blockDim.x) c += get(i) != 0xFFFFFFFFu;
    c = wave_sum_i32(c);
    if (lane_id() == 0) sh.red_i[wave_id()] = c;
    __syncthreads();
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) eq += sh.red_i[i];
    __syncthreads();
  }
  while (remaining > 0) {
    const int bits = remaining >= kDigitBits ? kDigitBits : remaining;
    const int nb = 1 << bits;
    const int shift = remaining - bits;
    const int top = shift + bits;
    for (int t = tid; t < nb; t += blockDim.x) sh.hist[t] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const uint32_t v = get(i);
      if (v == 0xFFFFFFFFu) continue;
      if (top < 32 && (v >> top) != prefix) continue;
      atomicAdd(&sh.hist[(v >> shift) & (uint32_t)(nb - 1)], 1);
    }
    __syncthreads();
    // each thread owns a run of per = nb / blockDim bins (at least one)
    const int per = (nb + blockDim.x - 1) / blockDim.x;
    const int b0 = tid * per;
    int mine = 0;
    for (int b = b0; b < min(nb, b0 + per); ++b) mine += sh.hist[b];
    const int incl = block_incl_scan(mine, sh.red_i);
    int excl = incl - mine;
    if (mine > 0 && excl < krem && krem <= incl) {
      for (int b = b0; b < min(nb, b0 + per); ++b) {
        const int c = sh.hist[b];
        if (excl + c >= krem) {
          sh.word = (prefix << bits) | (uint32_t)b;
          sh.krem = krem - excl;
          sh.eq = c;
          break;
        }
        excl += c;
      }
    }
    __syncthreads();
    prefix = sh.word;
    krem = sh.krem;
    eq = sh.eq;
    remaining -= bits;
    __syncthreads();
  }
  *krem_out = krem;
  *eq_out = eq;
  return prefix;
}

constexpr int kRowBatch = 8;    // survivor rows fetched together by one wave
constexpr int kEarlyKeys = 2048;  // keys requested before the count is known
constexpr int kRankSort = 256;  // entries up to which sort_pairs ranks instead of merging
constexpr int kCollectRounds = 8;  // positions per lane held in registers by the collect
constexpr bool kPairChunks = false;  // block kernel: two 256-value chunks of fp32 rows per round trip

// Sums over the wave of kRowBatch (8) values per lane at once: three halving
// exchanges (lanes 32 apart swap half of their values, then 16, then 8 apart)
// leave each lane one partial sum, of row 4 b5 + 2 b4 + b3 (bits of the lane
// index), which a butterfly over the 8 lanes of its group completes. 10
// exchanges instead of 48, in a fixed order; on return every lane holds the
// total of the row that its lane index names (lane >> 3).
template <int H, int O>
__device__ __forceinline__ void halve_rows(double (&acc)[kRowBatch], int lane) {
  const bool up = (lane & O) != 0;
#pragma unroll
  for (int r = 0; r < H; ++r) {
    const double keep = up ? acc[r + H] : acc[r];
    const double send = up ? acc[r] : acc[r + H];
    acc[r] = keep + (O >= 16 ? lane_xor_f64(send, O) : __shfl_xor(send, O));
  }
}

__device__ __forceinline__ double wave_sum8_f64(double (&acc)[kRowBatch]) {
  static_assert(kRowBatch == 8, "three halving steps");
  const int lane = lane_id();
  halve_rows<4, 32>(acc, lane);
  halve_rows<2, 16>(acc, lane);
  halve_rows<1, 8>(acc, lane);
  double v = acc[0];
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}

// FP64 partial sums of this lane for kRowBatch source rows: the sum of
// (q_i - d_i)^2 over the lane's values, chunk by chunk of 256 values (4
// consecutive per lane), in column order; wave_sum8_f64 then adds the lanes.
// With PAIR, fp32 rows of a length that is a multiple of 512 are fetched two
// chunks per round trip (more registers); otherwise one chunk at a time, and
// LEAN (1024-thread blocks, at most 128 VGPRs) fetches FP64 rows in halves.
// The sums are the same either way.
template <bool LEAN, bool PAIR>
__device__ __forceinline__ void rerank_batch(const SelRerankArgs &a, const float *qrow,
                                             const uint32_t (&row)[kRowBatch],
                                             double (&acc)[kRowBatch]) {
  const int lane = lane_id();
  const int nch = a.dp >> 8;    // chunks of 256 values: 4 per lane
  const int tail = a.dp & 255;  // remaining values (multiple of 16)
#pragma unroll
  for (int r = 0; r < kRowBatch; ++r) acc[r] = 0.0;
  if (PAIR && a.src32 && (a.dp & 511) == 0) {
    for (int c = 0; c < nch; c += 2) {
      const int col0 = c * 256 + lane * 4, col1 = col0 + 256;
      float4 y[2], v[2][kRowBatch];
      y[0] = *reinterpret_cast<const float4 *>(qrow + col0);
      y[1] = *reinterpret_cast<const float4 *>(qrow + col1);
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        const float *rp = a.src32 + (int64_t)row[r] * a.dp;
        v[0][r] = *reinterpret_cast<const float4 *>(rp + col0);
        v[1][r] = *reinterpret_cast<const float4 *>(rp + col1);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double y0 = y[h].x, y1 = y[h].y, y2 = y[h].z, y3 = y[h].w;
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
          double t;
          t = y0 - (double)v[h][r].x; acc[r] = fma(t, t, acc[r]);
          t = y1 - (double)v[h][r].y; acc[r] = fma(t, t, acc[r]);
          t = y2 - (double)v[h][r].z; acc[r] = fma(t, t, acc[r]);
          t = y3 - (double)v[h][r].w; acc[r] = fma(t, t, acc[r]);
        }
      }
    }
    return;
  }
  for (int c = 0; c <= nch; ++c) {
    const int col = c * 256 + lane * 4;
    if (c == nch && (tail == 0 || col >= a.dp)) break;
    const float4 y = *reinterpret_cast<const float4 *>(qrow + col);
    const double y0 = y.x, y1 = y.y, y2 = y.z, y3 = y.w;
    if (a.src32) {
      float4 v[kRowBatch];
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r)
        v[r] = *reinterpret_cast<const float4 *>(a.src32 + (int64_t)row[r] * a.dp + col);
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        double t;
        t = y0 - (double)v[r].x; acc[r] = fma(t, t, acc[r]);
        t = y1 - (double)v[r].y; acc[r] = fma(t, t, acc[r]);
        t = y2 - (double)v[r].z; acc[r] = fma(t, t, acc[r]);
        t = y3 - (double)v[r].w; acc[r] = fma(t, t, acc[r]);
      }
    } else if (LEAN) {
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        double2 v[kRowBatch];
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r)
          v[r] = reinterpret_cast<const double2 *>(a.src64 + (int64_t)row[r] * a.dp + col)[hf];
        const double ya = hf ? y2 : y0, yb = hf ? y3 : y1;
        __builtin_amdgcn_sched_barrier(0);  // keep the halves apart (register budget)
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
          double t;
          t = ya - v[r].x; acc[r] = fma(t, t, acc[r]);
          t = yb - v[r].y; acc[r] = fma(t, t, acc[r]);
        }
      }
    } else {
      double2 v[kRowBatch][2];
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        const double2 *rp = reinterpret_cast<const double2 *>(a.src64 + (int64_t)row[r] * a.dp + col);
        v[r][0] = rp[0];
        v[r][1] = rp[1];
      }
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        double t;
        t = y0 - v[r][0].x; acc[r] = fma(t, t, acc[r]);
        t = y1 - v[r][0].y; acc[r] = fma(t, t, acc[r]);
        t = y2 - v[r][1].x; acc[r] = fma(t, t, acc[r]);
        t = y3 - v[r][1].y; acc[r] = fma(t, t, acc[r]);
      }
    }
  }
}

// FP64 distances of the frame to source rows srow[s0 .. s1) into
// sort_hi / sort_lo[s] (distance bits, tie id); a kNoRow slot gets the key
// (kKeyNone, 0x80000000 | s), distinct and after every row. The calling
// wave takes the batches of kRowBatch rows starting at first, step apart;
// the tie ids are requested with the row values.
template <bool LEAN, bool PAIR>
__device__ void rerank_rows(const SelRerankArgs &a, const float *qrow, const uint32_t *srow,
                            uint64_t *sort_hi, uint32_t *sort_lo, int s1, int first, int step) {
  const int lane = lane_id();
  for (int b = first; b < s1; b += step) {
    uint32_t row[kRowBatch];
#pragma unroll
    for (int r = 0; r < kRowBatch; ++r) {
      const uint32_t v = srow[min(b + r, s1 - 1)];
      row[r] = v == kNoRow ? 0u : v;
    }
    // lanes 8 r .. 8 r + 7 end up holding row r's total
    const int sidx = b + (lane >> 3);
    const uint32_t rw = (lane & 7) == 0 && sidx < s1 ? srow[sidx] : kNoRow;
    const uint32_t tie = rw != kNoRow && a.tie_of ? (uint32_t)a.tie_of[rw] : rw;
    double acc[kRowBatch];
    rerank_batch<LEAN, PAIR>(a, qrow, row, acc);
    const double d = wave_sum8_f64(acc);
    if ((lane & 7) == 0 && sidx < s1) {
      if (rw == kNoRow) {
        sort_hi[sidx] = kKeyNone;
        sort_lo[sidx] = 0x80000000u | (uint32_t)sidx;
      } else {
        sort_hi[sidx] = (uint64_t)__double_as_longlong(d);
        sort_lo[sidx] = tie;
      }
    }
  }
}

// The block's waves share rows [s0, s1) of sh.srow, kRowBatch at a time.
template <bool LEAN>
__device__ void rerank_range(const SelRerankArgs &a, SelShared &sh, const float *qrow, int s0,
                             int s1) {
  const int w = wave_id(), nw = blockDim.x >> 6;
  rerank_rows<LEAN, kPairChunks && !LEAN>(a, qrow, sh.srow, sh.sort_hi, sh.sort_lo, s1,
                                          s0 + w * kRowBatch, nw * kRowBatch);
}

// Sorts hi / lo[0, cnt), cnt <= kWaveSort, by (hi, lo) in one wave: lane l
// holds entries l and l + 64 (empty ones past cnt) and a bitonic network
// exchanges them through shuffles, no barrier.
constexpr int kWaveSort = 128;
__device__ __forceinline__ bool pair_less(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah < bh || (ah == bh && al < bl);
}
__device__ void wave_sort_pairs128(uint64_t *hi, uint32_t *lo, int cnt) {
  const int lane = lane_id();
  uint64_t h[2];
  uint32_t l[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = lane + 64 * u;
    h[u] = e < cnt ? hi[e] : kKeyNone;
    l[u] = e < cnt ? lo[e] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int k = 2; k <= kWaveSort; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j == 64) {
        // partners in one lane (k = 128: ascending)
        if (pair_less(h[1], l[1], h[0], l[0])) {
          const uint64_t th = h[0];
          const uint32_t tl = l[0];
          h[0] = h[1];
          l[0] = l[1];
          h[1] = th;
          l[1] = tl;
        }
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint64_t ph = (uint64_t)__shfl_xor((long long)h[u], j);
          const uint32_t pl = (uint32_t)__shfl_xor((int)l[u], j);
          const int e = lane + 64 * u;
          // the lower element of an ascending pair (or the upper one of a
          // descending pair) keeps the smaller
          const bool keep_min = ((lane & j) == 0) == ((e & k) == 0);
          const bool p_less = pair_less(ph, pl, h[u], l[u]);
          if (keep_min == p_less) {
            h[u] = ph;
            l[u] = pl;
          }
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = lane + 64 * u;
    if (e < cnt) {
      hi[e] = h[u];
      lo[e] = l[u];
    }
  }
}

// Sorts sort_hi / sort_lo[0, cnt) ascending; the pairs are distinct (the
// second member is a candidate position or the tie id of a distinct row).
// Up to kWaveSort entries: wave_sort_pairs128 in the first wave. Up to
// kRankSort entries: G threads per entry (G consecutive lanes, G =
// blockDim / next_pow2(cnt), at most 64) each count the entries of a slice
// that order before it, the lanes add their counts and the entry is stored
// at that rank. Above, a bitonic merge in LDS over the entries padded to a
// power of two with empty ones.
__device__ void sort_pairs(SelShared &sh, int cnt) {
  const int tid = threadIdx.x;
  if (cnt <= kWaveSort) {
    __syncthreads();
    if (tid < 64) wave_sort_pairs128(sh.sort_hi, sh.sort_lo, cnt);
    __syncthreads();
    return;
  }
  if (cnt <= kRankSort && cnt <= (int)blockDim.x) {
    __syncthreads();
    const int G = min(64, (int)blockDim.x / next_pow2(max(cnt, 1)));
    const int e = tid / G, part = tid - e * G;
    uint64_t hi = 0;
    uint32_t lo = 0;
    int rank = 0;
    if (e < cnt) {
      hi = sh.sort_hi[e];
      lo = sh.sort_lo[e];
      const int per = (cnt + G - 1) / G, j0 = part * per, j1 = min(cnt, j0 + per);
      for (int j = j0; j < j1; j += 4) {
        uint64_t yh[4];
        uint32_t yl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int jj = min(j + u, j1 - 1);
          yh[u] = sh.sort_hi[jj];
          yl[u] = sh.sort_lo[jj];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          rank += (j + u < j1) & ((yh[u] < hi) | ((yh[u] == hi) & (yl[u] < lo)));
      }
    }
    for (int o = 1; o < G; o <<= 1) rank += __shfl_xor(rank, o);
    __syncthreads();
    if (e < cnt && part == 0) {
      sh.sort_hi[rank] = hi;
      sh.sort_lo[rank] = lo;
    }
    __syncthreads();
    return;
  }
  const int P = next_pow2(cnt);
  for (int t = cnt + tid; t < P; t += blockDim.x) {
    sh.sort_hi[t] = kKeyNone;
    sh.sort_lo[t] = 0xFFFFFFFFu;
  }
  block_sort_pairs(sh.sort_hi, sh.sort_lo, P);
}

// Entries [s, s + nb) (re-scored band rows, unsorted) merged into the sorted
// [0, s), s >= m: only band entries ordered before the m-th of [0, s) can
// enter the best m, so they are copied (through the select's histogram,
// free by now) behind the first m and those m + few are sorted;
// sort_hi / sort_lo[0, m) then hold the best m of all s + nb.
__device__ __noinline__ void merge_band(SelShared &sh, int s, int nb, int m) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const uint64_t mh = sh.sort_hi[m - 1];
  const uint32_t ml = sh.sort_lo[m - 1];
  auto before = [&](int t) {
    const uint64_t h = sh.sort_hi[t];
    return h < mh || (h == mh && sh.sort_lo[t] < ml);
  };
  int c = 0;
  for (int t = s + tid; t < s + nb; t += nt) c += before(t);
  const int incl = block_incl_scan(c, sh.red_i);
  if (tid == nt - 1) sh.eq = incl;
  int pos = incl - c;
  uint32_t *tmp = reinterpret_cast<uint32_t *>(sh.hist);  // 3 words per entry (nb <= 1024)
  for (int t = s + tid; t < s + nb; t += nt) {
    if (before(t)) {
      const uint64_t h = sh.sort_hi[t];
      tmp[3 * pos] = (uint32_t)h;
      tmp[3 * pos + 1] = (uint32_t)(h >> 32);
      tmp[3 * pos + 2] = sh.sort_lo[t];
      ++pos;
    }
  }
  __syncthreads();
  const int few = sh.eq;
  for (int i = tid; i < few; i += nt) {
    sh.sort_hi[m + i] = ((uint64_t)tmp[3 * i + 1] << 32) | tmp[3 * i];
    sh.sort_lo[m + i] = tmp[3 * i + 2];
  }
  sort_pairs(sh, m + few);  // (begins with a barrier)
}

// Source row of candidate position p of a frame: with region slots, slot j
// holds the rows from s_row[j] on at positions s_off[j] .. (s_off[0] = 0,
// non-decreasing; the slot holding p is the last with s_off[j] <= p, and it
// is never empty); without slots the position is the row.
__device__ __forceinline__ uint32_t row_of(const int32_t *s_off, const int32_t *s_row, int nslots,
                                           uint32_t p) {
  if (nslots == 0) return p;
  int lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_off[mid] <= (int32_t)p) lo = mid;
    else hi = mid;
  }
  return (uint32_t)(s_row[lo] + ((int32_t)p - s_off[lo]));
}

// Source row of row slot t (< kBlockRows) of block position p, or kNoRow
// past the block's last row: with region slots, slot j holds its region's
// blocks at positions s_off[j] .. (rows from s_row[j] on, s_len[j] of them);
// without, the block table of the exhaustive search.
__device__ __forceinline__ uint32_t block_row(const SelRerankArgs &a, const int32_t *s_off,
                                              const int32_t *s_row, const int32_t *s_len,
                                              int nslots, uint32_t p, int t) {
  int row0, len;
  if (nslots == 0) {
    const int2 br = a.blk_rows[p];
    row0 = br.x;
    len = br.y;
  } else {
    int lo = 0, hi = nslots;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= (int32_t)p) lo = mid;
      else hi = mid;
    }
    const int b = (int32_t)p - s_off[lo];
    row0 = s_row[lo] + b * kBlockRows;
    len = min(kBlockRows, s_len[lo] - b * kBlockRows);
  }
  return t < len ? (uint32_t)(row0 + t) : kNoRow;
}

// Source rows of positions sel[0 .. cnt) into srow[base ..): one per
// position, or kBlockRows per block position (kNoRow past a block's end).
__device__ __forceinline__ void positions_to_rows(const SelRerankArgs &a, SelShared &sh,
                                                  const int32_t *s_off, const int32_t *s_row,
                                                  const int32_t *s_len, int nslots, int cnt,
                                                  int base, const uint32_t *krow) {
  if (krow) {
    // key mode: the source row is the low half of the position's key
    for (int i = threadIdx.x; i < cnt; i += blockDim.x) sh.srow[base + i] = krow[sh.sel[i]];
  } else if (a.blocks) {
    for (int e = threadIdx.x; e < cnt * kBlockRows; e += blockDim.x) {
      const int i = e / kBlockRows, t = e - i * kBlockRows;
      sh.srow[base + e] = block_row(a, s_off, s_row, s_len, nslots, sh.sel[i], t);
    }
  } else {
    for (int i = threadIdx.x; i < cnt; i += blockDim.x)
      sh.srow[base + i] = row_of(s_off, s_row, nslots, sh.sel[i]);
  }
}

// Frame of block b in XCD-major order. Blocks go to the 8 XCDs round-robin
// (b % 8), so XCD x takes the contiguous run of frames starting at
// x * (n / 8) + min(x, n % 8): the frames of a request, which share most of
// their candidate rows, run on one XCD and share its L2.
__device__ __forceinline__ int xcd_frame(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, j = b / kXcd, q = n / kXcd, r = n % kXcd;
  return x * q + min(x, r) + j;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_select_rerank(SelRerankArgs a) {
  __shared__ SelShared sh;
  extern __shared__ uint32_t dyn[];  // [slot offsets | slot rows | slot sizes | word cache]
  if ((int)blockIdx.x >= a.nq) return;
  if (a.frame_list && (int)blockIdx.x >= *a.frame_count) return;
  const int f = a.frame_list ? a.frame_list[blockIdx.x] : xcd_frame(blockIdx.x, a.nq);
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  const int nw = blockDim.x >> 6;
  const int nslots = a.nslots;
  const int unit = a.blocks ? kBlockRows : 1;  // row slots per position
  int32_t *s_off = reinterpret_cast<int32_t *>(dyn);
  int32_t *s_row = s_off + nslots;
  int32_t *s_len = s_row + nslots;
  uint32_t *wc = dyn + 3 * nslots;
  const uint32_t *words = a.keys ? nullptr : a.cand + (int64_t)f * a.cap;
  // the first words are requested together with the count (one round trip)
  constexpr int EU = (kEarlyKeys + BLOCK - 1) / BLOCK;
  const int early = a.keys ? 0 : (int)min<int64_t>(a.cap, kEarlyKeys);
  uint32_t ew[EU];
#pragma unroll
  for (int u = 0; u < EU; ++u) {
    const int i = u * BLOCK + tid;
    ew[u] = i < early ? words[i] : kWordNone;
  }
  // the select's histogram and counter, cleared while the words are in flight
  static_assert((1 << kDigitBits) % (4 * BLOCK) == 0, "whole int4 per thread");
  for (int t = tid; t < (1 << kDigitBits) / 4; t += BLOCK)
    reinterpret_cast<int4 *>(sh.hist)[t] = make_int4(0, 0, 0, 0);
  if (tid == 0) sh.krem = 0;
  for (int j = tid; j < nslots; j += blockDim.x) {
    s_off[j] = a.slot_off[(int64_t)f * nslots + j];
    s_row[j] = a.slot_row[(int64_t)f * nslots + j];
    if (a.blocks) {
      s_len[j] = a.slot_len[(int64_t)f * nslots + j];
    }
  }
  const int n = a.n_cand ? a.n_cand[f] : a.n_fixed;
  // positions [0, C) cached, the rest read from memory (key mode: all, with
  // the keys' source rows behind the words)
  const int C = a.keys ? n : min(n, a.cache);
  uint32_t *krow = a.keys ? wc + n : nullptr;
  const float qn2 = a.qn2[f];
  auto word_at = [&](int i) -> uint32_t { return i < C ? wc[i] : words[i]; };

  int nv_local = 0;
  uint32_t vmin = 0xFFFFFFFFu, vmax = 0u;
  auto account = [&](int i, uint32_t v) {
    if (i >= n) return;
    if (i < C) wc[i] = v;
    if (v != kWordNone) {
      ++nv_local;
      vmin = min(vmin, v);
      vmax = max(vmax, v);
    }
  };
  uint64_t bmin = kKeyNone;  // key mode: smallest bound
  if (a.keys) {
    const uint64_t *kf = a.keys + (int64_t)f * n;
    for (int i = tid; i < n; i += blockDim.x) {
      const uint64_t kk = kf[i];
      account(i, (uint32_t)(kk >> 32));
      krow[i] = (uint32_t)kk;
    }
    const uint64_t *bf = a.bounds + (int64_t)f * a.n_bounds;
    for (int i = tid; i < a.n_bounds; i += blockDim.x) bmin = bf[i] < bmin ? bf[i] : bmin;
  } else {
#pragma unroll
    for (int u = 0; u < EU; ++u) account(u * BLOCK + tid, ew[u]);
    for (int base = EU * BLOCK; base < n; base += 8 * blockDim.x) {
      uint32_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int i = base + u * blockDim.x + tid;
        v[u] = i < n ? words[i] : kWordNone;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) account(base + u * blockDim.x + tid, v[u]);
    }
  }
  nv_local = wave_sum_i32(nv_local);
  vmin = wave_min_u32(vmin);
  vmax = wave_max_u32(vmax);
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t y = (uint64_t)__shfl_xor((long long)bmin, o);
    bmin = y < bmin ? y : bmin;
  }
  if (lane == 0) {
    sh.red_i[w] = nv_local;
    sh.red_u[w] = vmin;
    sh.red_v[w] = vmax;
    sh.red_k[w] = bmin;
  }
  __syncthreads();
  int nvalid = 0;
  vmin = 0xFFFFFFFFu;
  vmax = 0u;
  uint64_t bound = kKeyNone;
  for (int i = 0; i < nw; ++i) {
    nvalid += sh.red_i[i];
    vmin = min(vmin, sh.red_u[i]);
    vmax = max(vmax, sh.red_v[i]);
    bound = sh.red_k[i] < bound ? sh.red_k[i] : bound;
  }
  __syncthreads();
  const int L = a.L;
  const int nsurv = min(L, nvalid);
  const bool rejected = nvalid > L;
  // key mode: every source row missing from the keys has a word of at least
  // bw (the smallest of the frame's bounds); what the selection needs must
  // lie below it, else the frame is deferred to the dense screen
  const uint32_t bw = (uint32_t)(bound >> 32);
  // the frame goes to the dense screen instead (key mode, uniform over the
  // block); every later decision keeps that rule
  auto defer = [&]() {
    if (tid == 0) a.defer_list[atomicAdd(a.defer_count, 1)] = f;
  };
  if (bound != kKeyNone && !rejected) {
    defer();
    return;
  }
  // The L smallest (word, position) pairs become the survivors and the
  // (L+1)-th, (tw, tpos), the best rejected one: every rejected position has
  // a word above tw, or tw and a position from tpos on.
  uint32_t tw = kWordNone;
  int tpos = n;
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
  bool done = false;
  if (rejected && vmin != vmax) {
    // one histogram of the leading bits below the prefix shared by all
    // words; the words of the bucket holding the (L+1)-th and of every
    // bucket under it are then few: collect and sort them
    const int pre = __clz(vmin ^ vmax);
    const int bits = min(kDigitBits, 32 - pre), shift = 32 - pre - bits;
    const uint32_t mask = (1u << bits) - 1u;
    // (histogram and counter cleared at the start)
#pragma unroll 4
    for (int i = tid; i < n; i += BLOCK) {
      const uint32_t v = word_at(i);
      if (v != kWordNone) atomicAdd(&sh.hist[(v >> shift) & mask], 1);
    }
    __syncthreads();
    // each thread holds PB consecutive bins in registers (bins from 1 << bits
    // on are zero), scans their sums over the block and, if its run holds the
    // (L+1)-th word, finds the bucket there
    constexpr int PB = (1 << kDigitBits) / BLOCK;
    int hv[PB];
#pragma unroll
    for (int u = 0; u < PB; u += 4) {
      const int4 h = reinterpret_cast<const int4 *>(sh.hist + tid * PB)[u / 4];
      hv[u] = h.x;
      hv[u + 1] = h.y;
      hv[u + 2] = h.z;
      hv[u + 3] = h.w;
    }
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PB; ++u) mine += hv[u];
    const int incl = block_incl_scan(mine, sh.red_i);
    int excl = incl - mine;
    if (mine > 0 && excl < L + 1 && L + 1 <= incl) {
      bool found = false;
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        excl += hv[u];
        if (!found && excl >= L + 1) {
          found = true;
          sh.word = (uint32_t)(tid * PB + u);
          sh.eq = excl;  // words in buckets up to this one
        }
      }
    }
    __syncthreads();
    const uint32_t bstar = sh.word;
    const int m = sh.eq;
    if (m <= kMaxSurvivors) {
      // the words of buckets up to bstar, compacted by wave ballots: count,
      // one atomic per wave for its base, then place (any order). Up to
      // kCollectRounds positions per lane (half with 1024 threads) stay in
      // registers between the two.
      auto keep = [&](int i, uint32_t &v) {
        v = i < n ? word_at(i) : kWordNone;
        return v != kWordNone && ((v >> shift) & mask) <= bstar;
      };
      constexpr int CR = BLOCK >= 1024 ? kCollectRounds / 2 : kCollectRounds;
      if (n <= CR * BLOCK) {
        uint32_t v[CR];
        uint64_t bal[CR];
        int wcount = 0;
#pragma unroll
        for (int u = 0; u < CR; ++u) {
          bal[u] = __ballot(keep(u * BLOCK + w * 64 + lane, v[u]));
          wcount += __popcll(bal[u]);
        }
        int base = 0;
        if (lane == 0 && wcount > 0) base = atomicAdd(&sh.krem, wcount);
        base = __shfl(base, 0);
#pragma unroll
        for (int u = 0; u < CR; ++u) {
          if ((bal[u] >> lane) & 1ull) {
            const int slot = base + __popcll(bal[u] & ((1ull << lane) - 1ull));
            sh.sort_hi[slot] = v[u];
            sh.sort_lo[slot] = (uint32_t)(u * BLOCK + w * 64 + lane);
          }
          base += __popcll(bal[u]);
        }
      } else {
        // long lists (the exhaustive search: 200,000 words a frame): one
        // pass, one atomic per wave and 64 positions that keep any word
        // (few do), instead of a counting pass and a placing pass
        for (int b0 = w * 64; b0 < n; b0 += BLOCK) {
          uint32_t v;
          const bool k = keep(b0 + lane, v);
          const uint64_t bal = __ballot(k);
          if (bal) {
            int base = 0;
            if (lane == 0) base = atomicAdd(&sh.krem, __popcll(bal));
            base = __shfl(base, 0);
            if (k) {
              const int slot = base + __popcll(bal & ((1ull << lane) - 1ull));
              sh.sort_hi[slot] = v;
              sh.sort_lo[slot] = (uint32_t)(b0 + lane);
            }
          }
        }
      }
      __syncthreads();
      if (m == L + 1 && m <= BLOCK) {
        // usually: the (L+1)-th is the largest of the collected pairs (a
        // block maximum of word << 32 | position) and every other survives
        uint64_t key = 0;
        if (tid < m) key = (sh.sort_hi[tid] << 32) | sh.sort_lo[tid];
        uint64_t mx = key;
        for (int o = 32; o > 0; o >>= 1) {
          const uint64_t y = (uint64_t)__shfl_xor((long long)mx, o);
          mx = y > mx ? y : mx;
        }
        if (lane == 0) sh.red_k[w] = mx;
        __syncthreads();
        mx = 0;
        for (int i = 0; i < nw; ++i) mx = sh.red_k[i] > mx ? sh.red_k[i] : mx;
        if (tid < m && key == mx) sh.eq = tid;
        __syncthreads();
        const int imax = sh.eq;
        if (tid < m && key != mx) sh.sel[tid == L ? imax : tid] = (uint32_t)key;
        tw = (uint32_t)(mx >> 32);
        tpos = (int)(uint32_t)mx;
      } else {
        sort_pairs(sh, m);  // by (word, position)
        for (int t = tid; t < L; t += blockDim.x) sh.sel[t] = sh.sort_lo[t];
        tw = (uint32_t)sh.sort_hi[L];
        tpos = (int)sh.sort_lo[L];
      }
      __syncthreads();
      done = true;
    }
  }
  if (!done) {
    // radix select of the (L+1)-th word tw, then the survivors in position
    // order: every word below tw and the first take_eq positions whose word
    // equals tw (all valid words when none is rejected)
    int take_eq = 0;
    if (rejected) {
      int krem, eq;
      tw = block_select_u32(word_at, n, vmin, vmax, L + 1, sh, &krem, &eq);
      take_eq = krem - 1;
    }
    const int n_lt = nsurv - take_eq;
    int mlt = 0, meq = 0;
    for (int i = i0; i < i1; ++i) {
      const uint32_t v = word_at(i);
      mlt += v < tw;
      meq += rejected && v == tw;
    }
    int ilt = mlt, ieq = meq;
    block_incl_scan2(ilt, ieq, sh.red_i, sh.red_j);
    int plt = ilt - mlt, peq = ieq - meq;
    for (int i = i0; i < i1; ++i) {
      const uint32_t v = word_at(i);
      if (v < tw) {
        sh.sel[plt++] = (uint32_t)i;
      } else if (rejected && v == tw) {
        if (peq < take_eq) sh.sel[n_lt + peq] = (uint32_t)i;
        if (peq == take_eq) sh.krem = i;  // the first rejected position with word tw
        ++peq;
      }
    }
    __syncthreads();
    if (rejected) tpos = sh.krem;
    __syncthreads();
  }
  // key mode: the (L+1)-th word must not exceed what a list may have dropped
  if (rejected && bound != kKeyNone && tw > bw) {
    defer();
    return;
  }
  positions_to_rows(a, sh, s_off, s_row, s_len, nslots, nsurv, 0, krow);
  __syncthreads();
  // FP64 rerank of the survivors' rows, sorted by (distance, tie id); row
  // slots past a block's end sort last
  const int nrow = nsurv * unit;
  const float *qrow = a.qp + (int64_t)f * a.dp;
  rerank_range<BLOCK == 1024>(a, sh, qrow, 0, nrow);
  __syncthreads();
  sort_pairs(sh, nrow);
  // certificate: a rejected candidate can only beat the m-th reranked
  // distance dm if its screen distance is within the screen's error bound e
  // of dm. If the best rejected one is not beyond dm + e, every rejected
  // candidate up to dm + e (the band) is re-scored too, in chunks if it does
  // not fit at once. (In block mode a rejected block's word bounds all of its
  // rows from below; fewer than m rows so far make dm infinite.)
  if (tid == 0) {
    sh.flag = 0;
    if (rejected && a.m > 0) {
      const double rejd = (double)__uint_as_float(tw);
      const double qn = sqrt((double)qn2) * (1.0 + 1e-6);
      double e = a.err_coef * (qn + a.max_norm) * (qn + a.max_norm);
      if (a.q_err) {
        const double qe = a.q_err[f], ql = a.q_lon[f];
        e += a.lo_coef * (ql * a.lo_dmax + qe * a.lo_nmax + qe * a.lo_dmax);
      }
      const uint64_t km = sh.sort_hi[a.m - 1];
      const double dm = km == kKeyNone ? __builtin_inf() : __longlong_as_double((long long)km);
      const double tau = dm * (1.0 + 1e-12) + e;
      if (!(rejd > tau)) {
        sh.flag = 1;
        sh.word = __float_as_uint(__double2float_ru(tau));
        // key mode: a band reaching words the lists may have dropped is not
        // complete in the keys (flag 2: the frame is deferred)
        if (bound != kKeyNone && sh.word >= bw) sh.flag = 2;
        else if (a.stat_fallback) atomicAdd(a.stat_fallback, 1);
      }
    }
  }
  __syncthreads();
  int have = min(nrow, a.m);
  if (sh.flag == 2) {
    defer();
    return;
  }
  int band_rows = 0, fflags = 0;
  if (sh.flag == 1) {
    // the band: rejected positions (above tw, or equal to tw past the first
    // take_eq) with a word up to tau_w (>= tw)
    const uint32_t tau_w = sh.word;
    auto in_band = [&](uint32_t v, int i) {
      return v == tw ? i >= tpos : (v > tw && v <= tau_w);
    };
    int mine = 0;
    for (int i = i0; i < i1; ++i) mine += in_band(word_at(i), i);
    const int incl = block_incl_scan(mine, sh.red_i);
    __syncthreads();
    if (tid == blockDim.x - 1) sh.krem = incl;
    __syncthreads();
    const int total_band = sh.krem;
    // the survivors' positions are no longer needed: band positions go to
    // sel[0 ..), their rows behind the sorted survivor rows
    if (nrow + total_band * unit <= kMaxSurvivors) {
      int pos = incl - mine;
      for (int i = i0; i < i1; ++i)
        if (in_band(word_at(i), i)) sh.sel[pos++] = (uint32_t)i;
      __syncthreads();
      positions_to_rows(a, sh, s_off, s_row, s_len, nslots, total_band, nrow, krow);
      __syncthreads();
      rerank_range<BLOCK == 1024>(a, sh, qrow, nrow, nrow + total_band * unit);
      __syncthreads();
      merge_band(sh, nrow, total_band * unit, a.m);
      have = min(nrow + total_band * unit, a.m);
    } else {
      // a band too large for one pass: re-scored in chunks of up to
      // kMaxSurvivors - m rows, each merged with the best m so far (the
      // sorted survivors' first m to begin with). Every candidate that can
      // still enter the top m has a word up to tau_w, so this is exact.
      const int m = a.m, chunk = (kMaxSurvivors - m) / unit, excl = incl - mine;
      int kept = min(nrow, m);  // sort_hi / sort_lo[0, kept): the best so far, sorted
      fflags |= 2;
      for (int c0 = 0; c0 < total_band; c0 += chunk) {
        const int cnt = min(chunk, total_band - c0);
        // this thread's band positions ranked [c0, c0 + cnt) in position order
        __syncthreads();
        if (excl < c0 + cnt && excl + mine > c0) {
          int r = excl;
          for (int i = i0; i < i1 && r < c0 + cnt; ++i) {
            if (in_band(word_at(i), i)) {
              if (r >= c0) sh.sel[r - c0] = (uint32_t)i;
              ++r;
            }
          }
        }
        __syncthreads();
        positions_to_rows(a, sh, s_off, s_row, s_len, nslots, cnt, kept, krow);
        __syncthreads();
        rerank_range<BLOCK == 1024>(a, sh, qrow, kept, kept + cnt * unit);
        __syncthreads();
        merge_band(sh, kept, cnt * unit, m);
        kept = min(kept + cnt * unit, m);
      }
      have = kept;
    }
    band_rows = total_band * unit;
    fflags |= 1;
  }
  if (tid == 0 && a.frame_stat) a.frame_stat[f] = make_int4(n, nrow + band_rows, band_rows, fflags);
  for (int i = tid; i < a.m; i += blockDim.x) {
    const bool ok = i < have && sh.sort_hi[i] != kKeyNone;
    if (a.reg_out) {
      a.reg_out[(int64_t)f * a.m + i] = ok ? (int32_t)sh.sort_lo[i] : -1;
    } else {
      a.idx_out[(int64_t)f * a.m + i] = ok ? (int64_t)sh.sort_lo[i] : -1;
      a.dist_out[(int64_t)f * a.m + i] =
          ok ? (float)__longlong_as_double((long long)sh.sort_hi[i]) : __builtin_inff();
    }
  }
}

// Key mode in one wave per frame: the coarse stage after the fused coarse
// product when a frame has at most kWaveKeys keys. Its keys are few (the
// kept quads of each lane group and split), so a whole block per frame would
// mostly wait at barriers; here each wave takes one frame on its own (four
// frames per block, no block barrier) and follows the rules of
// k_select_rerank's key mode: the L smallest (word, position) pairs survive,
// the (L+1)-th decides the deferral and the certificate, the FP64 distances
// come from the same per-row arithmetic (rerank_rows), and the band is
// re-scored the same way, so the regions are the ones the block kernel
// would return. A band beyond kWaveRows rows defers the frame to the dense
// screen (exact as well).
constexpr int kWaveKeys = 256;  // keys per frame held by one wave (4 per lane)
constexpr int kWaveRows = 64;   // rows re-scored per frame by one wave
constexpr int kWaveFrames = 4;  // frames (waves) per block
struct WaveSel {
  uint32_t krow[kWaveKeys];     // source row of each key
  uint64_t sort_hi[kWaveRows];  // FP64 distance bits
  uint32_t sort_lo[kWaveRows];  // tie ids
  uint32_t srow[kWaveRows];     // rows to re-score
};

// Orders the wave's LDS accesses before and after (no block barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sorts sort_hi / sort_lo[0, cnt) (cnt <= 64, distinct pairs) by rank: lane t
// counts the entries ordered before entry t.
__device__ __forceinline__ void wave_sort_pairs(WaveSel &sh, int cnt) {
  const int lane = lane_id();
  uint64_t hi = kKeyNone;
  uint32_t lo = 0xFFFFFFFFu;
  int rank = 0;
  if (lane < cnt) {
    hi = sh.sort_hi[lane];
    lo = sh.sort_lo[lane];
    for (int j = 0; j < cnt; ++j) {
      const uint64_t yh = sh.sort_hi[j];
      const uint32_t yl = sh.sort_lo[j];
      rank += (yh < hi) | ((yh == hi) & (yl < lo));
    }
  }
  wave_sync();
  if (lane < cnt) {
    sh.sort_hi[rank] = hi;
    sh.sort_lo[rank] = lo;
  }
  wave_sync();
}

__global__ __launch_bounds__(64 * kWaveFrames) void k_select_keys(SelRerankArgs a) {
  __shared__ WaveSel s_all[kWaveFrames];
  const int w = wave_id(), lane = lane_id();
  const int ng = (a.nq + kWaveFrames - 1) / kWaveFrames;
  const int f = xcd_frame((int)blockIdx.x, ng) * kWaveFrames + w;
  if (f >= a.nq) return;  // (the whole wave; no block barrier follows)
  WaveSel &sh = s_all[w];
  const int n = a.n_fixed, L = a.L, m = a.m;
  constexpr int KPL = kWaveKeys / 64;  // keys per lane
  // the keys and bounds, requested together
  const uint64_t *kf = a.keys + (int64_t)f * n;
  uint64_t kk[KPL];
#pragma unroll
  for (int u = 0; u < KPL; ++u) {
    const int i = u * 64 + lane;
    kk[u] = i < n ? kf[i] : kKeyNone;
  }
  uint64_t bound = kKeyNone;
  for (int i = lane; i < a.n_bounds; i += 64) {
    const uint64_t b = a.bounds[(int64_t)f * a.n_bounds + i];
    bound = b < bound ? b : bound;
  }
  const float qn2 = a.qn2[f];
  // entries (word << 32 | position) of the valid keys (kKeyNone otherwise)
  uint64_t ent[KPL];
  int nv = 0;
#pragma unroll
  for (int u = 0; u < KPL; ++u) {
    const int i = u * 64 + lane;
    const uint32_t wd = (uint32_t)(kk[u] >> 32);
    const bool valid = i < n && wd != kWordNone;
    ent[u] = valid ? ((uint64_t)wd << 32) | (uint32_t)i : kKeyNone;
    sh.krow[i] = (uint32_t)kk[u];
    nv += valid;
  }
  const int nvalid = wave_sum_i32(nv);
  bound = wave_min_u64(bound);
  const bool rejected = nvalid > L;
  const uint32_t bw = (uint32_t)(bound >> 32);
  auto defer = [&]() {
    if (lane == 0) a.defer_list[atomicAdd(a.defer_count, 1)] = f;
  };
  if (bound != kKeyNone && !rejected) {
    defer();
    return;
  }
  // the survivors in (word, position) order: the wave minimum, taken out of
  // its lane, nsurv times; then the word tw of the best rejected pair
  // without taking it out
  const int nsurv = min(L, nvalid);
  wave_sync();  // krow written
  for (int t = 0; t < nsurv; ++t) {
    uint64_t lm = ent[0];
#pragma unroll
    for (int u = 1; u < KPL; ++u) lm = ent[u] < lm ? ent[u] : lm;
    const uint64_t mn = wave_min_u64(lm);
#pragma unroll
    for (int u = 0; u < KPL; ++u)
      if (ent[u] == mn) ent[u] = kKeyNone;
    if (lane == 0) sh.srow[t] = sh.krow[(uint32_t)mn];
  }
  uint32_t tw = kWordNone;
  if (rejected) {
    uint64_t lm = ent[0];
#pragma unroll
    for (int u = 1; u < KPL; ++u) lm = ent[u] < lm ? ent[u] : lm;
    tw = (uint32_t)(wave_min_u64(lm) >> 32);
  }
  if (rejected && bound != kKeyNone && tw > bw) {
    defer();
    return;
  }
  wave_sync();  // srow written
  const float *qrow = a.qp + (int64_t)f * a.dp;
  const int nrow = nsurv;
  rerank_rows<false, false>(a, qrow, sh.srow, sh.sort_hi, sh.sort_lo, nrow, 0, kRowBatch);
  wave_sync();
  wave_sort_pairs(sh, nrow);
  // certificate (the block kernel's, every lane alike)
  bool band = false;
  uint32_t tau_w = 0;
  if (rejected && m > 0) {
    const double rejd = (double)__uint_as_float(tw);
    const double qn = sqrt((double)qn2) * (1.0 + 1e-6);
    double e = a.err_coef * (qn + a.max_norm) * (qn + a.max_norm);
    if (a.q_err) {
      const double qe = a.q_err[f], ql = a.q_lon[f];
      e += a.lo_coef * (ql * a.lo_dmax + qe * a.lo_nmax + qe * a.lo_dmax);
    }
    const uint64_t km = sh.sort_hi[m - 1];
    const double dm = km == kKeyNone ? __builtin_inf() : __longlong_as_double((long long)km);
    const double tau = dm * (1.0 + 1e-12) + e;
    if (!(rejd > tau)) {
      band = true;
      tau_w = __float_as_uint(__double2float_ru(tau));
      // a band reaching words the lists may have dropped is not complete
      if (bound != kKeyNone && tau_w >= bw) {
        defer();
        return;
      }
    }
  }
  int have = min(nrow, m), band_rows = 0;
  if (band) {
    // the band: the pairs not taken out with a word up to tau_w (all of
    // them are at or after (tw, tpos)); their rows behind the survivors'
    int cnt[KPL], tot = 0;
#pragma unroll
    for (int u = 0; u < KPL; ++u) {
      const bool in = ent[u] != kKeyNone && (uint32_t)(ent[u] >> 32) <= tau_w;
      const uint64_t bal = __ballot(in);
      cnt[u] = in ? tot + __popcll(bal & ((1ull << lane) - 1ull)) : -1;
      tot += __popcll(bal);
    }
    if (nrow + tot > kWaveRows) {
      defer();
      return;
    }
#pragma unroll
    for (int u = 0; u < KPL; ++u)
      if (cnt[u] >= 0) sh.srow[nrow + cnt[u]] = sh.krow[(uint32_t)ent[u]];
    wave_sync();
    rerank_rows<false, false>(a, qrow, sh.srow, sh.sort_hi, sh.sort_lo, nrow + tot, nrow, kRowBatch);
    wave_sync();
    wave_sort_pairs(sh, nrow + tot);
    have = min(nrow + tot, m);
    band_rows = tot;
    if (lane == 0 && a.stat_fallback) atomicAdd(a.stat_fallback, 1);
  }
  if (lane == 0 && a.frame_stat)
    a.frame_stat[f] = make_int4(n, nrow + band_rows, band_rows, band ? 1 : 0);
  for (int i = lane; i < m; i += 64) {
    const bool ok = i < have && sh.sort_hi[i] != kKeyNone;
    a.reg_out[(int64_t)f * m + i] = ok ? (int32_t)sh.sort_lo[i] : -1;
  }
}

constexpr size_t select_lds_bytes(int nslots, int cache) {
  return (size_t)(3 * nslots + cache) * sizeof(uint32_t);
}
// the static block state plus the largest slot table and word cache fit the
// LDS one workgroup may hold
static_assert(sizeof(SelShared) + select_lds_bytes(kMaxSlots, kWordCache) <= (size_t)kLdsPerCu,
              "select kernel LDS above 160 KB");

// LDS limit of the select kernel (word cache and slot table above 64 KB),
// set once per device.
hipError_t prepare_select_kernels() {
  static int done_dev = -1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || done_dev == dev) return e;
  for (const void *k : {reinterpret_cast<const void *>(&k_select_rerank<256>),
                        reinterpret_cast<const void *>(&k_select_rerank<1024>)}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)select_lds_bytes(kMaxSlots, kWordCache));
    if (e != hipSuccess) return e;
  }
  if (e == hipSuccess) done_dev = dev;
  return e;
}

hipError_t launch_select_rerank(SelRerankArgs a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  const int unit = a.blocks ? kBlockRows : 1;
  if (a.L * unit > kMaxSurvivors || a.L * unit < a.m || a.m > 256) return hipErrorInvalidValue;
  if (a.frame_list && !a.frame_count) return hipErrorInvalidValue;
  if (a.nslots < 0 || a.nslots > kMaxSlots || (a.nslots > 0 && (!a.slot_off || !a.slot_row)))
    return hipErrorInvalidValue;
  if (a.blocks && ((a.nslots > 0 && !a.slot_len) ||
                   (a.nslots == 0 && !a.blk_rows)))
    return hipErrorInvalidValue;
  if (a.keys) {
    // key mode: every word and its source row cached, no slots, rows
    if (a.nslots != 0 || a.blocks || !a.bounds || a.n_bounds < 1 || a.cap != a.n_fixed ||
        2 * (int64_t)a.cap > kWordCache || !a.defer_list || !a.defer_count || a.frame_list)
      return hipErrorInvalidValue;
    a.cache = (int32_t)(2 * a.cap);
  } else {
    a.cache = (int32_t)std::min<int64_t>(a.cap, kWordCache);
  }
  // key mode with few keys per frame (the coarse stage of large batches):
  // one wave per frame
  if (a.keys && a.reg_out && a.n_fixed <= kWaveKeys && a.L <= kWaveRows)
    return launch_kernel(k_select_keys, dim3((unsigned)((a.nq + kWaveFrames - 1) / kWaveFrames)),
                         dim3(64 * kWaveFrames), 0, s, a);
  // frames with many candidates: the word cache takes most of the LDS, so the
  // block is alone on its compute unit; 1024 threads use all of it
  if (a.cap > kBigFrame)
    return launch_kernel(k_select_rerank<1024>, dim3(a.nq), dim3(1024),
                         (uint32_t)select_lds_bytes(a.nslots, a.cache), s, a);
  return launch_kernel(k_select_rerank<256>, dim3(a.nq), dim3(256),
                       (uint32_t)select_lds_bytes(a.nslots, a.cache), s, a);
}

}  // namespace hloc
