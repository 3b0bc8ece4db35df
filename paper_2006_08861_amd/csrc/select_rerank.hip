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
//      source rows through the frame's region slots, then FP64 direct sum of
//      (q_i - d_i)^2, ordered by (distance, tie id) with tie id = original row
//      index (fine stage) or region id (coarse stage);
//   3. certificate: the (L+1)-th word is the best rejected screen distance; if
//      it minus the screen's error bound does not exceed the m-th reranked
//      distance, the block also re-scores every rejected candidate within that
//      bound (or, if there are too many, all of them) and counts the frame.
// Distances are squared L2 (same order as the Euclidean distance of Section 4).
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

constexpr int kWordCache = 28672;  // screen words of a frame kept in (dynamic) LDS
constexpr int kBigFrame = 4096;    // candidate capacity above which a frame gets 1024 threads
constexpr int kMaxSlots = 1024;    // region slots of a frame kept in (dynamic) LDS
constexpr uint32_t kWordNone = 0xFFFFFFFFu;  // no candidate at this position
constexpr int kDigitBits = 12;     // radix digit of the select (two passes cover 24 bits)

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
  return v;
}
__device__ __forceinline__ int wave_sum_i32(int v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// FP64 squared distance of the padded fp32 frame to an FP64 source row, one
// wave; each lane sums its slice in order, then a fixed butterfly.
__device__ __forceinline__ double wave_dist_f64(const double *__restrict__ rp,
                                                const float *__restrict__ qrow, int dp) {
  const int lane = lane_id();
  double acc = 0.0;
  for (int c = lane * 2; c < dp; c += 128) {
    const double2 x = *reinterpret_cast<const double2 *>(rp + c);
    const float2 y = *reinterpret_cast<const float2 *>(qrow + c);
    double t;
    t = (double)y.x - x.x; acc = fma(t, t, acc);
    t = (double)y.y - x.y; acc = fma(t, t, acc);
  }
  return wave_sum_f64(acc);
}

// Sequential FP64 distance of one row (one thread; used by the fallback).
__device__ __forceinline__ double thread_dist(const SelRerankArgs &a, const float *qrow,
                                              uint32_t row) {
  double acc = 0.0;
  if (a.src64) {
    const double *rp = a.src64 + (int64_t)row * a.dp;
    for (int c = 0; c < a.dp; ++c) {
      const double t = (double)qrow[c] - rp[c];
      acc = fma(t, t, acc);
    }
  } else {
    const float *rp = a.src32 + (int64_t)row * a.dp;
    for (int c = 0; c < a.dp; ++c) {
      const double t = (double)qrow[c] - (double)rp[c];
      acc = fma(t, t, acc);
    }
  }
  return acc;
}

struct SelShared {
  uint32_t sel[kMaxSurvivors + 1];  // candidate positions of the survivors (+ band)
  uint32_t srow[kMaxSurvivors];     // their source rows
  uint64_t sort_hi[kMaxSurvivors];
  uint32_t sort_lo[kMaxSurvivors];
  int hist[1 << kDigitBits];
  int red_i[16];
  int red_j[16];
  uint32_t red_u[16];
  uint32_t red_v[16];
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

// Ascending bitonic sort of 64 (hi, lo) pairs, one per lane, by shuffles.
__device__ __forceinline__ void wave_sort64_pairs(uint64_t &hi, uint32_t &lo) {
  const int lane = lane_id();
  for (int size = 2; size <= 64; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint64_t ohi = (uint64_t)__shfl_xor((long long)hi, stride);
      const uint32_t olo = (uint32_t)__shfl_xor((int)lo, stride);
      const bool up = (lane & size) == 0;
      const bool lower = (lane & stride) == 0;
      const bool other_less = ohi < hi || (ohi == hi && olo < lo);
      const bool take = (lower == up) ? other_less : !other_less;
      if (take) {
        hi = ohi;
        lo = olo;
      }
    }
  }
}

constexpr int kRowBatch = 8;    // survivor rows fetched together by one wave
constexpr int kEarlyKeys = 1024;  // keys requested before the count is known

// FP64 distances of the frame to source rows sh.srow[s0 .. s1) into
// sort_hi / sort_lo[s] (distance bits, tie id). For fp32 sources each wave
// fetches kRowBatch rows at once with the frame slice reused across them.
__device__ void rerank_range(const SelRerankArgs &a, SelShared &sh, const float *qrow, int s0,
                             int s1) {
  const int w = wave_id(), lane = lane_id(), nw = blockDim.x >> 6;
  if (a.src32) {
    const int nch = a.dp >> 8;    // float4 chunks of 256 values per lane pass
    const int tail = a.dp & 255;  // remaining values (multiple of 32)
    for (int b = s0 + w * kRowBatch; b < s1; b += nw * kRowBatch) {
      double acc[kRowBatch];
      const float *rp[kRowBatch];
      uint32_t tie[kRowBatch];
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        acc[r] = 0.0;
        const uint32_t row = sh.srow[min(b + r, s1 - 1)];
        rp[r] = a.src32 + (int64_t)row * a.dp;
        tie[r] = (lane == r && a.tie_of) ? (uint32_t)a.tie_of[row] : row;
      }
      for (int c = 0; c <= nch; ++c) {
        const int col = c * 256 + lane * 4;
        if (c == nch && (tail == 0 || col >= a.dp)) break;
        const float4 y = *reinterpret_cast<const float4 *>(qrow + col);
        float4 x[kRowBatch];
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) x[r] = *reinterpret_cast<const float4 *>(rp[r] + col);
#pragma unroll
        for (int r = 0; r < kRowBatch; ++r) {
          double t;
          t = (double)y.x - (double)x[r].x; acc[r] = fma(t, t, acc[r]);
          t = (double)y.y - (double)x[r].y; acc[r] = fma(t, t, acc[r]);
          t = (double)y.z - (double)x[r].z; acc[r] = fma(t, t, acc[r]);
          t = (double)y.w - (double)x[r].w; acc[r] = fma(t, t, acc[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) acc[r] = wave_sum_f64(acc[r]);
#pragma unroll
      for (int r = 0; r < kRowBatch; ++r) {
        const int sidx = b + r;
        if (lane == r && sidx < s1) {
          sh.sort_hi[sidx] = (uint64_t)__double_as_longlong(acc[r]);
          sh.sort_lo[sidx] = tie[r];
        }
      }
    }
  } else {
    for (int sidx = s0 + w; sidx < s1; sidx += nw) {
      const uint32_t row = sh.srow[sidx];
      const double d = wave_dist_f64(a.src64 + (int64_t)row * a.dp, qrow, a.dp);
      if (lane == 0) {
        sh.sort_hi[sidx] = (uint64_t)__double_as_longlong(d);
        sh.sort_lo[sidx] = a.tie_of ? (uint32_t)a.tie_of[row] : row;
      }
    }
  }
}

// Sorts sort_hi / sort_lo[0, cnt) ascending (padding to a power of two with
// empty entries): by shuffles in one wave up to 64 entries, else in LDS.
__device__ void sort_pairs(SelShared &sh, int cnt) {
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  const int P = next_pow2(cnt > 0 ? cnt : 1);
  for (int t = cnt + tid; t < P; t += blockDim.x) {
    sh.sort_hi[t] = kKeyNone;
    sh.sort_lo[t] = 0xFFFFFFFFu;
  }
  __syncthreads();
  if (P <= 64) {
    if (w == 0) {
      uint64_t hi = lane < P ? sh.sort_hi[lane] : kKeyNone;
      uint32_t lo = lane < P ? sh.sort_lo[lane] : 0xFFFFFFFFu;
      wave_sort64_pairs(hi, lo);
      if (lane < P) {
        sh.sort_hi[lane] = hi;
        sh.sort_lo[lane] = lo;
      }
    }
    __syncthreads();
  } else {
    block_sort_pairs(sh.sort_hi, sh.sort_lo, P);
  }
}

// Source row of candidate position p of a frame: with region slots, slot j
// holds the rows of region s_reg[j] at positions s_off[j] .. (s_off[0] = 0,
// non-decreasing; the slot holding p is the last with s_off[j] <= p, and it
// is never empty); without slots the position is the row.
__device__ __forceinline__ uint32_t row_of(const int32_t *s_off, const int32_t *s_reg, int nslots,
                                           const int64_t *__restrict__ reg_start, uint32_t p) {
  if (nslots == 0) return p;
  int lo = 0, hi = nslots;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s_off[mid] <= (int32_t)p) lo = mid;
    else hi = mid;
  }
  return (uint32_t)(reg_start[s_reg[lo]] + ((int32_t)p - s_off[lo]));
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_select_rerank(SelRerankArgs a) {
  __shared__ SelShared sh;
  extern __shared__ uint32_t dyn[];  // [slot offsets | slot regions | word cache]
  const int f = blockIdx.x;
  if (f >= a.nq) return;
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  const int nw = blockDim.x >> 6;
  const int nslots = a.nslots;
  int32_t *s_off = reinterpret_cast<int32_t *>(dyn);
  int32_t *s_reg = s_off + nslots;
  uint32_t *wc = dyn + 2 * nslots;
  const uint32_t *words = a.cand + (int64_t)f * a.cap;
  // the first words are requested together with the count (one round trip)
  constexpr int EU = (kEarlyKeys + BLOCK - 1) / BLOCK;
  const int early = (int)min<int64_t>(a.cap, kEarlyKeys);
  uint32_t ew[EU];
#pragma unroll
  for (int u = 0; u < EU; ++u) {
    const int i = u * BLOCK + tid;
    ew[u] = i < early ? words[i] : kWordNone;
  }
  for (int j = tid; j < nslots; j += blockDim.x) {
    s_off[j] = a.slot_off[(int64_t)f * nslots + j];
    s_reg[j] = a.slot_reg[(int64_t)f * nslots + j];
  }
  const int n = a.n_cand ? a.n_cand[f] : a.n_fixed;
  const int C = min(n, a.cache);  // positions [0, C) cached, the rest read from memory
  const float qn2 = a.qn2[f];
  if (tid == 0 && a.stat_max) atomicMax(a.stat_max, n);
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
  nv_local = wave_sum_i32(nv_local);
  vmin = wave_min_u32(vmin);
  vmax = wave_max_u32(vmax);
  if (lane == 0) {
    sh.red_i[w] = nv_local;
    sh.red_u[w] = vmin;
    sh.red_v[w] = vmax;
  }
  __syncthreads();
  int nvalid = 0;
  vmin = 0xFFFFFFFFu;
  vmax = 0u;
  for (int i = 0; i < nw; ++i) {
    nvalid += sh.red_i[i];
    vmin = min(vmin, sh.red_u[i]);
    vmax = max(vmax, sh.red_v[i]);
  }
  __syncthreads();
  const int L = a.L;
  const int nsurv = min(L, nvalid);
  const bool rejected = nvalid > L;
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
    for (int t = tid; t < (1 << bits); t += blockDim.x) sh.hist[t] = 0;
    if (tid == 0) sh.krem = 0;
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) {
      const uint32_t v = word_at(i);
      if (v != kWordNone) atomicAdd(&sh.hist[(v >> shift) & mask], 1);
    }
    __syncthreads();
    const int nb = 1 << bits, pb = (nb + blockDim.x - 1) / blockDim.x, b0 = tid * pb;
    int mine = 0;
    for (int b = b0; b < min(nb, b0 + pb); ++b) mine += sh.hist[b];
    const int incl = block_incl_scan(mine, sh.red_i);
    int excl = incl - mine;
    if (mine > 0 && excl < L + 1 && L + 1 <= incl) {
      for (int b = b0; b < min(nb, b0 + pb); ++b) {
        excl += sh.hist[b];
        if (excl >= L + 1) {
          sh.word = (uint32_t)b;
          sh.eq = excl;  // words in buckets up to b
          break;
        }
      }
    }
    __syncthreads();
    const uint32_t bstar = sh.word;
    const int m = sh.eq;
    if (m <= kMaxSurvivors) {
      for (int i = i0; i < i1; ++i) {
        const uint32_t v = word_at(i);
        if (v != kWordNone && ((v >> shift) & mask) <= bstar) {
          const int slot = atomicAdd(&sh.krem, 1);
          sh.sort_hi[slot] = v;
          sh.sort_lo[slot] = (uint32_t)i;
        }
      }
      __syncthreads();
      sort_pairs(sh, m);  // by (word, position)
      for (int t = tid; t < L; t += blockDim.x) sh.sel[t] = sh.sort_lo[t];
      tw = (uint32_t)sh.sort_hi[L];
      tpos = (int)sh.sort_lo[L];
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
  for (int s = tid; s < nsurv; s += blockDim.x)
    sh.srow[s] = row_of(s_off, s_reg, nslots, a.reg_start, sh.sel[s]);
  __syncthreads();
  // FP64 rerank of the survivors, sorted by (distance, tie id)
  const float *qrow = a.qp + (int64_t)f * a.dp;
  rerank_range(a, sh, qrow, 0, nsurv);
  __syncthreads();
  sort_pairs(sh, nsurv);
  // certificate: a rejected candidate can only beat the m-th reranked
  // distance dm if its screen distance is within the screen's error bound e
  // of dm. If the best rejected one is not beyond dm + e, every rejected
  // candidate up to dm + e (the band) is re-scored too; if the band does not
  // fit, every candidate is.
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
      const double dm = __longlong_as_double((long long)sh.sort_hi[a.m - 1]);
      const double tau = dm * (1.0 + 1e-12) + e;
      if (!(rejd > tau)) {
        sh.flag = 1;
        sh.word = __float_as_uint(__double2float_ru(tau));
        if (a.stat_fallback) atomicAdd(a.stat_fallback, 1);
      }
    }
  }
  __syncthreads();
  int have = min(nsurv, a.m);
  if (sh.flag) {
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
    if (nsurv + total_band <= kMaxSurvivors) {
      int pos = nsurv + incl - mine;
      for (int i = i0; i < i1; ++i)
        if (in_band(word_at(i), i)) sh.sel[pos++] = (uint32_t)i;
      __syncthreads();
      for (int s = nsurv + tid; s < nsurv + total_band; s += blockDim.x)
        sh.srow[s] = row_of(s_off, s_reg, nslots, a.reg_start, sh.sel[s]);
      __syncthreads();
      rerank_range(a, sh, qrow, nsurv, nsurv + total_band);
      __syncthreads();
      sort_pairs(sh, nsurv + total_band);
      have = min(nsurv + total_band, a.m);
    } else {
      // exact FP64 top m over every candidate, merged 256 at a time into a
      // sorted best list held in sort_hi / sort_lo[0, Pm)
      const int Pm = next_pow2(a.m);
      const int Q = next_pow2(Pm + 256);
      for (int t = tid; t < Q; t += blockDim.x) {
        sh.sort_hi[t] = kKeyNone;
        sh.sort_lo[t] = 0xFFFFFFFFu;
      }
      for (int base = 0; base < n; base += 256) {
        const int i = base + tid;
        uint64_t hi = kKeyNone;
        uint32_t lo = 0xFFFFFFFFu;
        if (i < n && tid < 256) {
          if (word_at(i) != kWordNone) {
            const uint32_t row = row_of(s_off, s_reg, nslots, a.reg_start, (uint32_t)i);
            hi = (uint64_t)__double_as_longlong(thread_dist(a, qrow, row));
            lo = a.tie_of ? (uint32_t)a.tie_of[row] : row;
          }
        }
        __syncthreads();
        for (int t = Pm + tid; t < Q; t += blockDim.x) {
          sh.sort_hi[t] = kKeyNone;
          sh.sort_lo[t] = 0xFFFFFFFFu;
        }
        __syncthreads();
        if (tid < 256) {
          sh.sort_hi[Pm + tid] = hi;
          sh.sort_lo[Pm + tid] = lo;
        }
        block_sort_pairs(sh.sort_hi, sh.sort_lo, Q);
      }
      have = min(nvalid, a.m);
    }
  }
  for (int i = tid; i < a.m; i += blockDim.x) {
    const bool ok = i < have;
    if (a.reg_out) {
      a.reg_out[(int64_t)f * a.m + i] = ok ? (int32_t)sh.sort_lo[i] : -1;
    } else {
      a.idx_out[(int64_t)f * a.m + i] = ok ? (int64_t)sh.sort_lo[i] : -1;
      a.dist_out[(int64_t)f * a.m + i] =
          ok ? (float)__longlong_as_double((long long)sh.sort_hi[i]) : __builtin_inff();
    }
  }
}

size_t select_lds_bytes(int nslots, int cache) {
  return (size_t)(2 * nslots + cache) * sizeof(uint32_t);
}

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
  if (a.L > kMaxSurvivors || a.L < a.m || a.m > 256) return hipErrorInvalidValue;
  if (a.nslots < 0 || a.nslots > kMaxSlots || (a.nslots > 0 && (!a.slot_off || !a.slot_reg)))
    return hipErrorInvalidValue;
  a.cache = (int32_t)std::min<int64_t>(a.cap, kWordCache);
  // frames with many candidates: the word cache takes most of the LDS, so the
  // block is alone on its compute unit; 1024 threads use all of it
  if (a.cap > kBigFrame)
    return launch_kernel(k_select_rerank<1024>, dim3(a.nq), dim3(1024),
                         (uint32_t)select_lds_bytes(a.nslots, a.cache), s, a);
  return launch_kernel(k_select_rerank<256>, dim3(a.nq), dim3(256),
                       (uint32_t)select_lds_bytes(a.nslots, a.cache), s, a);
}

}  // namespace hloc
