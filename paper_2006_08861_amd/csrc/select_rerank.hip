// Top candidates per frame ("select top candidates", Algorithm 1), one block
// per frame, in one kernel:
//   1. select: the L + 1 smallest screen keys (dist_bits << 32 | row; one
//      integer compare orders by screen distance, then row). The keys are
//      cached in LDS; a radix select finds the distance word of the (L+1)-th
//      key (leading bits shared by the smallest and largest word skipped, the
//      rest resolved 8 bits per pass with an LDS histogram), a second one its
//      row among the keys with that word. Keys are unique, so exactly L + 1
//      keys are <= the threshold;
//   2. rerank: FP64 direct sum of (q_i - d_i)^2 for the L smallest (the
//      survivors), ordered by (distance, tie id) with tie id = original row
//      index (fine stage) or region id (coarse stage);
//   3. certificate: the largest selected key is the best rejected screen
//      distance; if it minus the screen's error bound does not exceed the
//      m-th reranked distance, the block also re-scores every rejected
//      candidate within that bound (or, if there are too many, all of them)
//      and counts the frame.
// Distances are squared L2 (same order as the Euclidean distance of Section 4).
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

constexpr int kKeyCache = 8192;  // candidate keys kept in (dynamic) LDS

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
  uint64_t sel[kMaxSurvivors + 1];
  uint64_t sort_hi[kMaxSurvivors];
  uint32_t sort_lo[kMaxSurvivors];
  int hist[4096];
  int part[256];
  int red_i[16];
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

// Block-wide radix select over 32-bit words: returns the target-th smallest
// (1-based) of get(i), i < n, ignoring 0xFFFFFFFF (no candidate); every other
// word lies in [lo, hi]. *krem_out receives its rank among equal words and
// *eq_out how many words equal it. Leading bits shared by lo and hi are
// skipped; the rest are resolved 12 bits per pass with an LDS histogram.
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
    const int bits = remaining >= 12 ? 12 : remaining;
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

// FP64 distances of the frame to source rows sh.sel[s0 .. s1) into
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
        const uint32_t row = (uint32_t)sh.sel[min(b + r, s1 - 1)];
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
      const uint32_t row = (uint32_t)sh.sel[sidx];
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

__global__ __launch_bounds__(256) void k_select_rerank(SelRerankArgs a) {
  __shared__ SelShared sh;
  extern __shared__ uint64_t kc[];  // up to kKeyCache keys of the frame
  const int f = blockIdx.x;
  if (f >= a.nq) return;
  const int tid = threadIdx.x, w = wave_id(), lane = lane_id();
  const int nw = blockDim.x >> 6;
  const uint64_t *keys = a.cand + (int64_t)f * a.cap;
  // the first keys are requested together with the count (one round trip)
  const int early = (int)min<int64_t>(a.cap, kEarlyKeys);
  uint64_t ek[kEarlyKeys / 256];
#pragma unroll
  for (int u = 0; u < kEarlyKeys / 256; ++u) {
    const int i = u * 256 + tid;
    ek[u] = (i < early && tid < 256) ? keys[i] : kKeyNone;
  }
  const int n = a.n_cand ? a.n_cand[f] : a.n_fixed;
  const float qn2 = a.qn2[f];
  const bool cached = n <= kKeyCache;
  if (tid == 0 && a.stat_max) atomicMax(a.stat_max, n);
  auto key_at = [&](int i) -> uint64_t { return cached ? kc[i] : keys[i]; };

  int nv_local = 0;
  uint32_t vmin = 0xFFFFFFFFu, vmax = 0u;
  auto account = [&](int i, uint64_t k) {
    if (i >= n) return;
    if (cached) kc[i] = k;
    if (k != kKeyNone) {
      const uint32_t h = (uint32_t)(k >> 32);
      ++nv_local;
      vmin = min(vmin, h);
      vmax = max(vmax, h);
    }
  };
#pragma unroll
  for (int u = 0; u < kEarlyKeys / 256; ++u) account(u * 256 + tid, ek[u]);
  for (int base = kEarlyKeys; base < n; base += 4 * blockDim.x) {
    uint64_t k[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = base + u * blockDim.x + tid;
      k[u] = i < n ? keys[i] : kKeyNone;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) account(base + u * blockDim.x + tid, k[u]);
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
  // the (L+1)-th smallest key: its distance word by radix select, then, if
  // several keys share that word, its row among them
  uint64_t thresh = kKeyNone;
  if (rejected) {
    int krem, eq;
    const uint32_t tw = block_select_u32([&](int i) { return (uint32_t)(key_at(i) >> 32); }, n,
                                         vmin, vmax, L + 1, sh, &krem, &eq);
    uint32_t rw;
    if (eq == 1) {
      // the one key with word tw: found by whichever thread holds it
      for (int i = tid; i < n; i += blockDim.x) {
        const uint64_t k = key_at(i);
        if ((uint32_t)(k >> 32) == tw) sh.word = (uint32_t)k;
      }
      __syncthreads();
      rw = sh.word;
      __syncthreads();
    } else {
      int e2;
      rw = block_select_u32(
          [&](int i) {
            const uint64_t k = key_at(i);
            return (uint32_t)(k >> 32) == tw ? (uint32_t)k : 0xFFFFFFFFu;
          },
          n, 0u, 0x7FFFFFFFu, krem, sh, &krem, &e2);
    }
    thresh = ((uint64_t)tw << 32) | rw;
  }
  // survivors: every valid key below the threshold (all valid keys if none is
  // rejected); each thread takes a contiguous run, one block scan places them
  {
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int i0 = tid * per, i1 = min(n, i0 + per);
    int mine = 0;
    for (int i = i0; i < i1; ++i) {
      const uint64_t k = key_at(i);
      mine += k != kKeyNone && k < thresh;
    }
    int pos = block_incl_scan(mine, sh.red_i) - mine;
    for (int i = i0; i < i1; ++i) {
      const uint64_t k = key_at(i);
      if (k != kKeyNone && k < thresh) sh.sel[pos++] = k;
    }
    __syncthreads();
  }
  // FP64 rerank of the survivors, sorted by (distance, tie id)
  const float *qrow = a.qp + (int64_t)f * a.dp;
  rerank_range(a, sh, qrow, 0, nsurv);
  __syncthreads();
  sort_pairs(sh, nsurv);
  // certificate: a rejected key can only beat the m-th reranked distance dm if
  // its screen distance is within the screen's error bound e of dm. If the
  // best rejected one is not beyond dm + e, every rejected key up to dm + e
  // (the band) is re-scored too; if the band does not fit, every candidate is.
  if (tid == 0) {
    sh.flag = 0;
    if (rejected && a.m > 0) {
      const double rejd = (double)__uint_as_float((uint32_t)(thresh >> 32));
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
    const uint32_t tau_w = sh.word;
    const int per = (n + blockDim.x - 1) / blockDim.x;
    const int i0 = tid * per, i1 = min(n, i0 + per);
    int mine = 0;
    for (int i = i0; i < i1; ++i) {
      const uint64_t k = key_at(i);
      mine += k != kKeyNone && k >= thresh && (uint32_t)(k >> 32) <= tau_w;
    }
    const int incl = block_incl_scan(mine, sh.red_i);
    __syncthreads();
    if (tid == blockDim.x - 1) sh.krem = incl;
    __syncthreads();
    const int total_band = sh.krem;
    if (nsurv + total_band <= kMaxSurvivors) {
      int pos = nsurv + incl - mine;
      for (int i = i0; i < i1; ++i) {
        const uint64_t k = key_at(i);
        if (k != kKeyNone && k >= thresh && (uint32_t)(k >> 32) <= tau_w) sh.sel[pos++] = k;
      }
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
        if (i < n) {
          const uint64_t k = key_at(i);
          if (k != kKeyNone) {
            const uint32_t row = (uint32_t)k;
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

// LDS limit of the select kernel (key cache above 64 KB), set once per device.
hipError_t prepare_select_kernels() {
  static int done_dev = -1;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || done_dev == dev) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_select_rerank),
                          hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(kKeyCache * sizeof(uint64_t)));
  if (e == hipSuccess) done_dev = dev;
  return e;
}

hipError_t launch_select_rerank(const SelRerankArgs &a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (a.L > kMaxSurvivors || a.L < a.m || a.m > 256) return hipErrorInvalidValue;
  const size_t lds = (size_t)kKeyCache * sizeof(uint64_t);
  return launch_kernel(k_select_rerank, dim3(a.nq), dim3(256), lds, s, a);
}

}  // namespace hloc
