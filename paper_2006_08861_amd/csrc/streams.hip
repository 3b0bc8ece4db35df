// Sliding windows across calls (Section 3.1: a request for frame q_m carries
// the frames before it; M = 11 in Section 4). A video stream sends each frame
// once; the library keeps, per stream, the top-k lists of its last M - 1
// frames on the device, so the window of a new frame pools M lists of which
// only the new frame's is retrieved.
//
// Layout of the state's list buffer: S x (M - 1) history lists (stream s,
// oldest first, `count[s]` of them valid), then room for the new frames of
// one call. A call retrieves its new frames straight into that room, builds
// each new frame's window as a list of indices into the buffer, aggregates
// the windows (Algorithm 2, the frame list form of the aggregation kernel)
// and then moves each stream's last M - 1 lists to the stream's history.
#include <new>

#include "hloc_device.h"
#include "hloc_host.h"

struct hloc_streams {
  hloc_db *db = nullptr;
  hloc_ws *ws = nullptr;   // workspace of the retrieval
  int32_t S = 0, M = 0, k = 0, max_frames = 0;
  int64_t *lists = nullptr;       // (S (M - 1) + max_frames) x k
  int32_t *count = nullptr;       // S: valid history lists per stream
  int32_t *last_call = nullptr;   // S: 2 x the last call with a segment of the stream (+1: several)
  int32_t *win_off = nullptr;     // max_frames + 1
  int32_t *win_list = nullptr;    // max_frames x M
  int32_t *seg_ok = nullptr;      // max_frames: segments of a call that passed the checks
  float *dist = nullptr;          // max_frames x k (when the caller wants no distances)
  int32_t call = 0;               // calls so far
};

namespace hloc {
namespace {

constexpr int kStreamThreads = 1024;

// Segment (of the call's segments) holding new frame j: the last g with
// seg_off[g] <= j.
__device__ __forceinline__ int segment_of(const int32_t *seg_off, int nseg, int j) {
  int lo = 0, hi = nseg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg_off[mid] <= j) lo = mid;
    else hi = mid;
  }
  return lo;
}

// One block. Each segment (a run of new frames of one stream, in capture
// order) is checked first: its stream must lie in [0, S) and be the stream of
// no other segment of this call. Then every new frame's window: the last
// from_hist history lists of its stream, the new frames of its segment before
// it (at most M - 1 together) and itself; a frame of a rejected segment gets
// the one-entry list {-1}, which the aggregation flags HLOC_FLAG_BAD_REQUEST.
__global__ __launch_bounds__(kStreamThreads) void k_stream_windows(
    const int32_t *seg_off, const int32_t *seg_stream, int nseg, int nq, int S, int M,
    int call, const int32_t *count, int32_t *last_call, int32_t *seg_ok, int32_t *win_off,
    int32_t *win_list) {
  __shared__ int s_tot[kStreamThreads / 64];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
  // last_call[s] only grows: 2 call once a segment of s is seen in this
  // call, 2 call + 1 once a second one is
  for (int g = tid; g < nseg; g += blockDim.x) {
    const int s = seg_stream[g];
    if (s >= 0 && s < S && atomicMax(&last_call[s], 2 * call) == 2 * call)
      atomicMax(&last_call[s], 2 * call + 1);
  }
  __threadfence();  // the marks are complete before any is read
  __syncthreads();
  for (int g = tid; g < nseg; g += blockDim.x) {
    const int s = seg_stream[g];
    const bool ranged = seg_off[g] >= 0 && seg_off[g] <= seg_off[g + 1] && seg_off[g + 1] <= nq;
    seg_ok[g] = ranged && s >= 0 && s < S && atomicOr(&last_call[s], 0) == 2 * call;
  }
  if (tid == 0) s_base = 0;
  __syncthreads();
  const int H = M - 1;
  for (int j0 = 0; j0 < nq; j0 += blockDim.x) {
    const int j = j0 + tid;
    int g = 0, len = 0, from_hist = 0, from_new = 0, s = 0;
    bool ok = false;
    if (j < nq) {
      g = segment_of(seg_off, nseg, j);
      ok = seg_ok[g] && j >= seg_off[g] && j < seg_off[g + 1];
      if (ok) {
        s = seg_stream[g];
        from_new = min(j - seg_off[g], H);
        from_hist = min(count[s], H - from_new);
        len = from_hist + from_new + 1;
      } else {
        len = 1;
      }
    }
    // exclusive scan of the lengths over the block, in frame order
    int inc = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (lane == 63) s_tot[w] = inc;
    __syncthreads();
    int before = s_base;
    for (int i = 0; i < w; ++i) before += s_tot[i];
    const int off = before + inc - len;
    if (j < nq) {
      win_off[j] = off;
      if (!ok) {
        win_list[off] = -1;
      } else {
        int p = off;
        const int c = count[s];
        for (int h = c - from_hist; h < c; ++h) win_list[p++] = s * H + h;
        for (int i = j - from_new; i <= j; ++i) win_list[p++] = S * H + i;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int t = s_base;
      for (int i = 0; i < nw; ++i) t += s_tot[i];
      s_base = t;
    }
    __syncthreads();
  }
  if (tid == 0) win_off[nq] = s_base;
}

// One block per segment: the stream's new history is the last M - 1 lists of
// (its history, its new frames); the lists that stay are read before any is
// written.
__global__ __launch_bounds__(256) void k_stream_update(const int32_t *seg_off,
                                                       const int32_t *seg_stream,
                                                       const int32_t *seg_ok, int S, int M, int k,
                                                       int64_t *lists, int32_t *count) {
  extern __shared__ int64_t s_keep[];  // (M - 1) x k
  const int g = blockIdx.x;
  if (!seg_ok[g]) return;
  const int s = seg_stream[g], H = M - 1;
  const int nnew = seg_off[g + 1] - seg_off[g];
  const int c = count[s];
  const int take_new = min(nnew, H);
  const int keep_old = min(c, H - take_new);
  int64_t *hist = lists + (int64_t)s * H * k;
  const int64_t *fresh = lists + ((int64_t)S * H + seg_off[g] + nnew - take_new) * k;
  for (int t = threadIdx.x; t < (keep_old + take_new) * k; t += blockDim.x) {
    const int h = t / k, i = t - h * k;
    s_keep[t] = h < keep_old ? hist[(int64_t)(c - keep_old + h) * k + i]
                             : fresh[(int64_t)(h - keep_old) * k + i];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (keep_old + take_new) * k; t += blockDim.x) hist[t] = s_keep[t];
  if (threadIdx.x == 0) count[s] = keep_old + take_new;
}

__global__ void k_fill_i32_s(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void destroy(hloc_streams *st) {
  if (!st) return;
  for (void *p : {static_cast<void *>(st->lists), static_cast<void *>(st->count),
                  static_cast<void *>(st->last_call), static_cast<void *>(st->win_off),
                  static_cast<void *>(st->win_list), static_cast<void *>(st->seg_ok),
                  static_cast<void *>(st->dist)})
    if (p) (void)hipFree(p);
  if (st->ws) {
    --st->db->user_ws;
    free_ws(st->ws);
  }
  delete st;
}

}  // namespace
}  // namespace hloc

using namespace hloc;

extern "C" {

int hloc_streams_create(hloc_db *db, int32_t n_streams, int32_t window, int32_t k,
                        int32_t max_frames, hloc_streams **out) {
  if (!out) return fail(HLOC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (n_streams < 1) return fail(HLOC_EINVAL, "n_streams must be >= 1 (got %d)", n_streams);
  if (k < 1 || k > HLOC_MAX_K) return fail(HLOC_EINVAL, "k must be in 1..%d (got %d)", HLOC_MAX_K, k);
  if (window < 1 || (int64_t)window * k > HLOC_MAX_REQUEST_CANDIDATES)
    return fail(HLOC_EINVAL, "window must be >= 1 with window x k <= %d (got %d x %d)",
                HLOC_MAX_REQUEST_CANDIDATES, window, k);
  if (max_frames < 1) return fail(HLOC_EINVAL, "max_frames must be >= 1 (got %d)", max_frames);
  const int64_t H = window - 1;
  if ((int64_t)n_streams * H + max_frames > INT32_MAX / 2)
    return fail(HLOC_EINVAL, "n_streams x (window - 1) + max_frames is too large");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  hloc_streams *st = new (std::nothrow) hloc_streams();
  if (!st) return fail(HLOC_ENOMEM, "host allocation failed");
  st->db = db;
  st->S = n_streams;
  st->M = window;
  st->k = k;
  st->max_frames = max_frames;
  const int64_t nlists = (int64_t)n_streams * H + max_frames;
  bool ok = hipMalloc(&st->lists, (size_t)nlists * k * sizeof(int64_t)) == hipSuccess &&
            hipMalloc(&st->count, (size_t)n_streams * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&st->last_call, (size_t)n_streams * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&st->win_off, (size_t)(max_frames + 1) * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&st->win_list, (size_t)max_frames * window * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&st->seg_ok, (size_t)max_frames * sizeof(int32_t)) == hipSuccess &&
            hipMalloc(&st->dist, (size_t)max_frames * k * sizeof(float)) == hipSuccess;
  if (!ok) {
    destroy(st);
    return fail(HLOC_ENOMEM, "device allocation of the stream state failed");
  }
  int rc = new_ws(db, &st->ws);
  if (rc != HLOC_OK) {
    st->ws = nullptr;
    destroy(st);
    return rc;
  }
  ++db->user_ws;
  const int grid = (n_streams + 255) / 256;
  if (launch_kernel(k_fill_i32_s, dim3(grid), dim3(256), 0, st->ws->stream, st->count,
                    (int64_t)n_streams, 0) != hipSuccess ||
      launch_kernel(k_fill_i32_s, dim3(grid), dim3(256), 0, st->ws->stream, st->last_call,
                    (int64_t)n_streams, -1) != hipSuccess ||
      hipStreamSynchronize(st->ws->stream) != hipSuccess) {
    destroy(st);
    return fail(HLOC_EDEVICE, "clearing the stream state failed");
  }
  *out = st;
  return HLOC_OK;
}

int hloc_streams_reset(hloc_streams *st) {
  if (!st) return fail(HLOC_EINVAL, "st is NULL");
  DeviceGuard g(st->db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(launch_kernel(k_fill_i32_s, dim3((st->S + 255) / 256), dim3(256), 0, st->ws->stream,
                       st->count, (int64_t)st->S, 0));
  HIPCHK(hipStreamSynchronize(st->ws->stream));
  return HLOC_OK;
}

void hloc_streams_free(hloc_streams *st) {
  if (!st) return;
  DeviceGuard g(st->db->device);
  (void)hipDeviceSynchronize();
  destroy(st);
}

int hloc_query_streams_async(hloc_streams *st, const float *q, int32_t nq, int32_t n_regions,
                             int32_t precision, const int32_t *seg_offsets,
                             const int32_t *seg_stream, int32_t nseg, int64_t *idx, float *dist,
                             double *xy, int32_t *tile, int32_t *flags, void *stream) {
  if (!st) return fail(HLOC_EINVAL, "st is NULL");
  hloc_db *db = st->db;
  if (nq < 0 || nq > st->max_frames)
    return fail(HLOC_EINVAL, "nq must be in 0..%d (got %d)", st->max_frames, nq);
  if (nseg < 0 || nseg > nq) return fail(HLOC_EINVAL, "nseg must be in 0..nq (got %d)", nseg);
  if (nq > 0 && (!q || !seg_offsets || !seg_stream || !xy || !tile || !flags))
    return fail(HLOC_EINVAL, "q, seg_offsets, seg_stream, xy, tile and flags must be non-NULL");
  if (nq > 0 && nseg < 1) return fail(HLOC_EINVAL, "frames need at least one segment");
  if ((idx == nullptr) != (dist == nullptr))
    return fail(HLOC_EINVAL, "idx and dist are both given or both NULL");
  Plan p;
  CHK(make_plan(db, nq, st->k, n_regions, nq, precision, &p));  // nq windows
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  if (nq == 0) return HLOC_OK;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int32_t S = st->S, M = st->M, k = st->k, H = M - 1;
  // the new frames' lists go straight behind the histories
  int64_t *fresh = st->lists + (int64_t)S * H * k;
  CHK(enqueue_query(st->ws, p, q, nullptr, nullptr, fresh, dist ? dist : st->dist, nullptr,
                    nullptr, nullptr, s));
  ++st->call;
  int32_t *seg_ok = st->seg_ok;
  HIPCHK(launch_kernel(k_stream_windows, dim3(1), dim3(kStreamThreads), 0, s, seg_offsets,
                       seg_stream, nseg, nq, S, M, st->call, st->count, st->last_call, seg_ok,
                       st->win_off, st->win_list));
  AggArgs ag{};
  ag.idx = st->lists;
  ag.k = k;
  ag.nq = S * H + nq;
  ag.req_offsets = st->win_off;
  ag.nreq = nq;
  ag.tile_of = db->tiles;
  ag.cell = db->cell;
  ag.top_c = db->top_c;
  ag.rho = db->rho;
  ag.toler_pct = db->pct;
  ag.xy = xy;
  ag.tile = tile;
  ag.flags = flags;
  ag.big_list = as<int32_t>(st->ws->agg_big);
  ag.big_count = as<int32_t>(st->ws->misc) + 8;  // cleared by the retrieval's prep kernel
  ag.num_cu = db->num_cu;
  HIPCHK(launch_aggregate_frames(ag, st->win_list, (int32_t)std::min<int64_t>(
                                     (int64_t)nq * M, INT32_MAX), s));
  if (H > 0)
    HIPCHK(launch_kernel(k_stream_update, dim3(nseg), dim3(256),
                         (uint32_t)((size_t)H * k * sizeof(int64_t)), s, seg_offsets, seg_stream,
                         seg_ok, S, M, k, st->lists, st->count));
  if (idx)
    HIPCHK(hipMemcpyAsync(idx, fresh, (size_t)nq * k * sizeof(int64_t), hipMemcpyDeviceToDevice,
                          s));
  return HLOC_OK;
}

}  // extern "C"
