// Top candidates per frame ("select top candidates", Algorithm 1) in three
// steps:
//   select : the `want` smallest screen keys of a frame (packed
//            dist_bits << 32 | row, so one integer compare orders by screen
//            distance then row);
//   rerank : FP64 direct sum of (q_i - d_i)^2 for the want - 1 survivors,
//            ordered by (distance, tie id), and a certificate: the best
//            rejected screen distance minus the screen's error bound must
//            exceed the m-th reranked distance, otherwise the frame is flagged;
//   exact  : for flagged frames only, FP64 distances over the frame's whole
//            candidate set and an exact top-m.
// Distances are squared L2 (same order as the Euclidean distance of Section 4);
// ties go to the smaller original row index.
#include "hloc_device.h"
#include "hloc_internal.h"

namespace hloc {

__global__ __launch_bounds__(256) void k_select(const uint64_t *__restrict__ cand, int64_t cap,
                                                const int32_t *__restrict__ n_cand, int n_fixed,
                                                int nq, int want, uint64_t *__restrict__ sel,
                                                int32_t *stat_max) {
  __shared__ uint64_t buf[kSelectLds];
  __shared__ int scratch[16];
  const int f = blockIdx.x;
  if (f >= nq) return;
  const int tid = threadIdx.x;
  const int n = n_cand ? n_cand[f] : n_fixed;
  const uint64_t *src = cand + (int64_t)f * cap;
  uint64_t *dst = sel + (int64_t)f * want;
  if (tid == 0 && stat_max) atomicMax(stat_max, n);
  if (n <= kSelectLds) {
    const int p = next_pow2(n > 0 ? n : 1);
    for (int i = tid; i < p; i += blockDim.x) buf[i] = i < n ? src[i] : kKeyNone;
    block_sort_u64(buf, p);
    for (int i = tid; i < want; i += blockDim.x) dst[i] = i < n ? buf[i] : kKeyNone;
    return;
  }
  // Streaming selection: the best P keys sit sorted in buf[0, P); keys below
  // the current P-th best are appended after them and the whole buffer is
  // re-sorted when it fills.
  const int P = next_pow2(want);
  const int room = kSelectLds - P;
  for (int i = tid; i < kSelectLds; i += blockDim.x) buf[i] = src[i];
  block_sort_u64(buf, kSelectLds);
  uint64_t tau = buf[P - 1];
  int cnt = 0;
  for (int base = kSelectLds; base < n; base += blockDim.x) {
    const int i = base + tid;
    const uint64_t key = i < n ? src[i] : kKeyNone;
    bool pass = key < tau;
    int tot;
    int pos = block_excl_count(pass, scratch, &tot);
    if (cnt + tot > room) {
      for (int t = P + cnt + tid; t < kSelectLds; t += blockDim.x) buf[t] = kKeyNone;
      block_sort_u64(buf, kSelectLds);
      tau = buf[P - 1];
      cnt = 0;
      pass = key < tau;
      pos = block_excl_count(pass, scratch, &tot);
    }
    if (pass) buf[P + cnt + pos] = key;
    cnt += tot;
  }
  for (int t = P + cnt + tid; t < kSelectLds; t += blockDim.x) buf[t] = kKeyNone;
  block_sort_u64(buf, kSelectLds);
  for (int i = tid; i < want; i += blockDim.x) dst[i] = buf[i];
}

hipError_t launch_select(const uint64_t *cand, int64_t cap, const int32_t *n_cand,
                         int32_t n_fixed, int32_t nq, int32_t want, uint64_t *sel,
                         int32_t *stat_max, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  if (next_pow2_host(want) > kSelectLds / 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select, dim3(nq), dim3(256), 0, s, cand, cap, n_cand, n_fixed, nq, want,
                     sel, stat_max);
  return hipGetLastError();
}

// FP64 squared distance of frame row qrow (fp32, padded) to source row; each
// lane sums its slice in order, then a fixed butterfly; lane 0 has the value.
__device__ __forceinline__ double wave_dist_f32(const float *__restrict__ rp,
                                                const float *__restrict__ qrow, int dp) {
  const int lane = lane_id();
  double acc = 0.0;
  for (int c = lane * 4; c < dp; c += 256) {
    const float4 x = *reinterpret_cast<const float4 *>(rp + c);
    const float4 y = *reinterpret_cast<const float4 *>(qrow + c);
    double t;
    t = (double)y.x - (double)x.x; acc = fma(t, t, acc);
    t = (double)y.y - (double)x.y; acc = fma(t, t, acc);
    t = (double)y.z - (double)x.z; acc = fma(t, t, acc);
    t = (double)y.w - (double)x.w; acc = fma(t, t, acc);
  }
  return wave_sum_f64(acc);
}

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

__global__ __launch_bounds__(256) void k_rerank(RerankArgs a) {
  __shared__ uint64_t s_hi[kMaxSurvivors];
  __shared__ uint32_t s_lo[kMaxSurvivors];
  __shared__ int s_nv;
  const int f = blockIdx.x;
  if (f >= a.nq) return;
  const int tid = threadIdx.x, wave = wave_id(), lane = lane_id();
  const int n = a.n_cand ? a.n_cand[f] : a.n_fixed;
  const uint64_t *sel = a.sel + (int64_t)f * a.want;
  const int L = a.want - 1;
  if (tid == 0) s_nv = 0;
  __syncthreads();
  int mine = 0;
  for (int t = tid; t < L; t += blockDim.x) mine += sel[t] != kKeyNone;
  if (mine) atomicAdd(&s_nv, mine);
  __syncthreads();
  const int nv = s_nv;  // sel is sorted, so the survivors are sel[0, nv)
  const int P = next_pow2(nv > 0 ? nv : 1);
  const float *qrow = a.qp + (int64_t)f * a.dp;
  for (int sidx = wave; sidx < nv; sidx += 4) {
    const uint32_t row = (uint32_t)sel[sidx];
    const double d = a.src32 ? wave_dist_f32(a.src32 + (int64_t)row * a.dp, qrow, a.dp)
                             : wave_dist_f64(a.src64 + (int64_t)row * a.dp, qrow, a.dp);
    if (lane == 0) {
      s_hi[sidx] = (uint64_t)__double_as_longlong(d);
      s_lo[sidx] = a.tie_of ? (uint32_t)a.tie_of[row] : row;
    }
  }
  for (int t = nv + tid; t < P; t += blockDim.x) {
    s_hi[t] = kKeyNone;
    s_lo[t] = 0xFFFFFFFFu;
  }
  block_sort_pairs(s_hi, s_lo, P);
  for (int i = tid; i < a.m; i += blockDim.x) {
    const bool ok = i < nv;
    if (a.reg_out) {
      a.reg_out[(int64_t)f * a.m + i] = ok ? (int32_t)s_lo[i] : -1;
    } else {
      a.idx_out[(int64_t)f * a.m + i] = ok ? (int64_t)s_lo[i] : -1;
      a.dist_out[(int64_t)f * a.m + i] =
          ok ? (float)__longlong_as_double((long long)s_hi[i]) : __builtin_inff();
    }
  }
  if (tid == 0) {
    bool certified = true;
    if (n > L && nv >= a.m && a.m > 0) {
      const uint64_t rej = sel[L];
      if (rej != kKeyNone) {
        const double rejd = (double)__uint_as_float((uint32_t)(rej >> 32));
        const double qn = sqrt((double)a.qn2[f]) * (1.0 + 1e-6);
        const double e = a.err_coef * (qn + a.max_norm) * (qn + a.max_norm);
        const double dm = __longlong_as_double((long long)s_hi[a.m - 1]);
        certified = (rejd - e) > dm * (1.0 + 1e-12);
      }
    }
    a.flag[f] = certified ? 0 : 1;
    if (!certified && a.stat_fallback) atomicAdd(a.stat_fallback, 1);
  }
}

hipError_t launch_rerank(const RerankArgs &a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (a.want - 1 > kMaxSurvivors || a.m > a.want - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rerank, dim3(a.nq), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Exact FP64 top-m over the whole candidate set of each flagged frame. One
// thread per candidate, chunks of 256 merged into a running sorted best list.
__global__ __launch_bounds__(256) void k_exact(ExactArgs a) {
  __shared__ uint64_t s_hi[512];
  __shared__ uint32_t s_lo[512];
  const int f = blockIdx.x;
  if (f >= a.nq || a.flag[f] == 0) return;
  const int tid = threadIdx.x;
  const int P = next_pow2(a.m);
  const int Q = next_pow2(P + 256);
  const float *qrow = a.qp + (int64_t)f * a.dp;
  const int total = a.src64 ? a.R : a.n_cand[f];
  const int32_t *coff = a.src64 ? nullptr : a.cand_off + (int64_t)f * a.nr;
  for (int t = tid; t < P; t += blockDim.x) {
    s_hi[t] = kKeyNone;
    s_lo[t] = 0xFFFFFFFFu;
  }
  for (int base = 0; base < total; base += 256) {
    const int p = base + tid;
    uint64_t hi = kKeyNone;
    uint32_t lo = 0xFFFFFFFFu;
    if (p < total) {
      if (a.src64) {
        if (a.reg_start[p + 1] > a.reg_start[p]) {
          const double *rp = a.src64 + (int64_t)p * a.dp;
          double acc = 0.0;
          for (int c = 0; c < a.dp; ++c) {
            const double t = (double)qrow[c] - rp[c];
            acc = fma(t, t, acc);
          }
          hi = (uint64_t)__double_as_longlong(acc);
          lo = (uint32_t)p;
        }
      } else {
        // last kept region whose first position is <= p (empty regions
        // have equal offsets; the last of them is the non-empty owner)
        int lo_j = 0, hi_j = a.nr - 1;
        while (lo_j < hi_j) {
          const int mid = (lo_j + hi_j + 1) >> 1;
          if (coff[mid] <= p) lo_j = mid; else hi_j = mid - 1;
        }
        const int r = a.regions[(int64_t)f * a.nr + lo_j];
        const int64_t row = a.reg_start[r] + (p - coff[lo_j]);
        const float *rp = a.src32 + row * a.dp;
        double acc = 0.0;
        for (int c = 0; c < a.dp; ++c) {
          const double t = (double)qrow[c] - (double)rp[c];
          acc = fma(t, t, acc);
        }
        hi = (uint64_t)__double_as_longlong(acc);
        lo = (uint32_t)a.tie_of[row];
      }
    }
    __syncthreads();
    for (int t = P + tid; t < Q; t += blockDim.x) {
      s_hi[t] = kKeyNone;
      s_lo[t] = 0xFFFFFFFFu;
    }
    __syncthreads();
    s_hi[P + tid] = hi;
    s_lo[P + tid] = lo;
    block_sort_pairs(s_hi, s_lo, Q);
  }
  for (int i = tid; i < a.m; i += blockDim.x) {
    const bool ok = s_hi[i] != kKeyNone;
    if (a.src64) {
      a.reg_out[(int64_t)f * a.m + i] = ok ? (int32_t)s_lo[i] : -1;
    } else {
      a.idx_out[(int64_t)f * a.m + i] = ok ? (int64_t)s_lo[i] : -1;
      a.dist_out[(int64_t)f * a.m + i] =
          ok ? (float)__longlong_as_double((long long)s_hi[i]) : __builtin_inff();
    }
  }
}

hipError_t launch_exact(const ExactArgs &a, hipStream_t s) {
  if (a.nq <= 0) return hipSuccess;
  if (a.m > 256) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_exact, dim3(a.nq), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace hloc
