// Request server: continuous batching of localization requests over one
// database, the client/server request model of Section 3.1 (a request brings
// the frames around one position; the answer is each frame's top-N
// candidates and one floor-plan position, Section 3.2).
//
// Requests wait in a FIFO queue. A launcher thread takes the oldest waiting
// requests that fit one batch (never splitting a request) whenever one of the
// slots is free, packs their frames into the slot's pinned staging buffer and
// enqueues copy-in, the whole query path and copy-out on the slot's stream; a
// completion thread waits for the slots in launch order and hands each
// request its rows of the batch's results. Up to `slots` batches overlap on
// the device while new requests arrive. Every slot is sized for a full batch
// when the server is created, so serving allocates no device memory.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hloc_host.h"

using namespace hloc;

namespace {

using Clock = std::chrono::steady_clock;

enum { kQueued = 0, kRunning = 1, kDone = 2, kFailed = 3 };

struct Request {
  uint64_t ticket = 0;
  int32_t nframes = 0, k = 0;
  std::vector<float> frames;  // nframes x d
  std::vector<int64_t> idx;   // nframes x k
  std::vector<float> dist;    // nframes x k
  double xy[2] = {0.0, 0.0};
  int32_t tile[2] = {0, 0};
  int32_t flags = 0;
  int state = kQueued;
  Clock::time_point t_submit, t_done;
};

// One batch in flight: its workspace (and stream), pinned staging on the
// host and input/output buffers on the device, all sized for a full batch.
struct Slot {
  hloc_ws *ws = nullptr;
  float *h_q = nullptr;
  int32_t *h_off = nullptr, *h_k = nullptr;
  int64_t *h_idx = nullptr;
  float *h_dist = nullptr;
  double *h_xy = nullptr;
  int32_t *h_tile = nullptr, *h_flags = nullptr;
  float *d_q = nullptr;
  int32_t *d_off = nullptr, *d_k = nullptr;
  int64_t *d_idx = nullptr;
  float *d_dist = nullptr;
  double *d_xy = nullptr;
  int32_t *d_tile = nullptr, *d_flags = nullptr;
  hipEvent_t done = nullptr;
  std::vector<Request *> reqs;
  int32_t nq = 0;
  bool busy = false;
};

}  // namespace

struct hloc_server {
  hloc_db *db = nullptr;
  hloc_server_config cfg{};
  size_t slot_bytes = 0;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_launch, cv_complete, cv_done;
  std::deque<Request *> queue;
  std::deque<int> inflight;  // slot ids in launch order
  std::unordered_map<uint64_t, Request *> reqs;
  uint64_t next_ticket = 1;
  int64_t queued_frames = 0;
  bool stop = false;
  int err_code = HLOC_OK;
  std::string err_msg;
  std::thread launcher, completer;
  int64_t st_batches = 0, st_requests = 0, st_frames = 0, st_max_batch = 0, st_peak_queue = 0,
          st_max_inflight = 0, st_refused = 0;
};

namespace {

// Device bytes of the input/output buffers of a batch of F frames.
size_t io_bytes(const hloc_db *db, int32_t F, int32_t k) {
  return alloc_size((size_t)F * db->d * sizeof(float)) + 2 * alloc_size((size_t)(F + 1) * sizeof(int32_t)) +
         alloc_size((size_t)F * k * sizeof(int64_t)) + alloc_size((size_t)F * k * sizeof(float)) +
         alloc_size((size_t)F * 2 * sizeof(double)) + alloc_size((size_t)F * 2 * sizeof(int32_t)) +
         alloc_size((size_t)F * sizeof(int32_t));
}

template <class T>
int slot_alloc(T **dev, T **host, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  if (hipMalloc(reinterpret_cast<void **>(dev), alloc_size(bytes)) != hipSuccess) {
    (void)hipGetLastError();
    *dev = nullptr;
    return fail(HLOC_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  if (host && hipHostMalloc(reinterpret_cast<void **>(host), bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    *host = nullptr;
    return fail(HLOC_ENOMEM, "pinned host allocation of %zu bytes failed", bytes);
  }
  return HLOC_OK;
}

void free_slot(Slot &s) {
  for (void *p : {(void *)s.d_q, (void *)s.d_off, (void *)s.d_k, (void *)s.d_idx, (void *)s.d_dist,
                  (void *)s.d_xy, (void *)s.d_tile, (void *)s.d_flags})
    if (p) (void)hipFree(p);
  for (void *p : {(void *)s.h_q, (void *)s.h_off, (void *)s.h_k, (void *)s.h_idx, (void *)s.h_dist,
                  (void *)s.h_xy, (void *)s.h_tile, (void *)s.h_flags})
    if (p) (void)hipHostFree(p);
  if (s.done) (void)hipEventDestroy(s.done);
  free_ws(s.ws);
  s = Slot{};
}

int make_slot(hloc_server *srv, const Plan &full, Slot &s) {
  hloc_db *db = srv->db;
  const int32_t F = srv->cfg.max_batch_frames, k = srv->cfg.k;
  CHK(new_ws(db, &s.ws));
  CHK(ensure_workspace(s.ws, full, false));
  CHK(slot_alloc(&s.d_q, &s.h_q, (size_t)F * db->d));
  CHK(slot_alloc(&s.d_off, &s.h_off, (size_t)F + 1));
  CHK(slot_alloc(&s.d_k, &s.h_k, (size_t)F + 1));
  CHK(slot_alloc(&s.d_idx, &s.h_idx, (size_t)F * k));
  CHK(slot_alloc(&s.d_dist, &s.h_dist, (size_t)F * k));
  CHK(slot_alloc(&s.d_xy, &s.h_xy, (size_t)F * 2));
  CHK(slot_alloc(&s.d_tile, &s.h_tile, (size_t)F * 2));
  CHK(slot_alloc(&s.d_flags, &s.h_flags, (size_t)F));
  HIPCHK(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
  return HLOC_OK;
}

// Enqueues copy-in, the query path and copy-out of the slot's requests on the
// slot's stream, then records s.done.
int launch_batch(hloc_server *srv, Slot &s) {
  hloc_db *db = srv->db;
  const int32_t d = db->d, k = srv->cfg.k;
  const int32_t nreq = (int32_t)s.reqs.size();
  int32_t nq = 0;
  s.h_off[0] = 0;
  for (int32_t j = 0; j < nreq; ++j) {
    const Request *r = s.reqs[j];
    std::memcpy(s.h_q + (size_t)nq * d, r->frames.data(), (size_t)r->nframes * d * sizeof(float));
    nq += r->nframes;
    s.h_off[j + 1] = nq;
    s.h_k[j] = r->k;
  }
  s.nq = nq;
  Plan p;
  CHK(make_plan(db, nq, k, srv->cfg.n_regions, nreq, srv->cfg.precision, &p));
  hipStream_t st = s.ws->stream;
  HIPCHK(hipMemcpyAsync(s.d_q, s.h_q, (size_t)nq * d * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s.d_off, s.h_off, (size_t)(nreq + 1) * sizeof(int32_t),
                        hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(s.d_k, s.h_k, (size_t)nreq * sizeof(int32_t), hipMemcpyHostToDevice, st));
  CHK(enqueue_query(s.ws, p, s.d_q, s.d_off, s.d_k, s.d_idx, s.d_dist, s.d_xy, s.d_tile,
                    s.d_flags, st));
  HIPCHK(hipMemcpyAsync(s.h_idx, s.d_idx, (size_t)nq * k * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s.h_dist, s.d_dist, (size_t)nq * k * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s.h_xy, s.d_xy, (size_t)nreq * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s.h_tile, s.d_tile, (size_t)nreq * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(s.h_flags, s.d_flags, (size_t)nreq * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipEventRecord(s.done, st));
  return HLOC_OK;
}

int free_slot_id(const hloc_server *srv) {
  for (size_t i = 0; i < srv->slots.size(); ++i)
    if (!srv->slots[i].busy) return (int)i;
  return -1;
}

void launcher_main(hloc_server *srv) {
  (void)hipSetDevice(srv->db->device);
  const int32_t F = srv->cfg.max_batch_frames;
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    srv->cv_launch.wait(lk, [&] {
      return srv->stop || (srv->err_code == HLOC_OK && !srv->queue.empty() && free_slot_id(srv) >= 0);
    });
    if (srv->stop) return;
    const int si = free_slot_id(srv);
    Slot &s = srv->slots[si];
    s.reqs.clear();
    int32_t nq = 0;
    while (!srv->queue.empty() && nq + srv->queue.front()->nframes <= F) {
      Request *r = srv->queue.front();
      srv->queue.pop_front();
      nq += r->nframes;
      srv->queued_frames -= r->nframes;
      r->state = kRunning;
      s.reqs.push_back(r);
    }
    s.busy = true;
    lk.unlock();
    const int rc = launch_batch(srv, s);
    const std::string msg = rc == HLOC_OK ? std::string() : std::string(hloc_last_error());
    lk.lock();
    if (rc != HLOC_OK) {
      for (Request *r : s.reqs) r->state = kFailed;
      s.reqs.clear();
      s.busy = false;
      srv->err_code = rc;
      srv->err_msg = msg;
      srv->cv_done.notify_all();
      continue;
    }
    srv->inflight.push_back(si);
    srv->st_max_inflight = std::max<int64_t>(srv->st_max_inflight, (int64_t)srv->inflight.size());
    srv->cv_complete.notify_one();
  }
}

void completer_main(hloc_server *srv) {
  (void)hipSetDevice(srv->db->device);
  const int32_t k = srv->cfg.k;
  std::unique_lock<std::mutex> lk(srv->mu);
  for (;;) {
    srv->cv_complete.wait(lk, [&] { return srv->stop || !srv->inflight.empty(); });
    if (srv->inflight.empty()) return;  // stop requested and nothing in flight
    Slot &s = srv->slots[srv->inflight.front()];
    lk.unlock();
    const hipError_t e = hipEventSynchronize(s.done);
    if (e == hipSuccess) {
      int32_t f = 0;
      for (size_t j = 0; j < s.reqs.size(); ++j) {
        Request *r = s.reqs[j];
        r->idx.resize((size_t)r->nframes * r->k);
        r->dist.resize((size_t)r->nframes * r->k);
        for (int32_t i = 0; i < r->nframes; ++i) {
          std::memcpy(&r->idx[(size_t)i * r->k], s.h_idx + (size_t)(f + i) * k, r->k * sizeof(int64_t));
          std::memcpy(&r->dist[(size_t)i * r->k], s.h_dist + (size_t)(f + i) * k, r->k * sizeof(float));
        }
        r->xy[0] = s.h_xy[2 * j];
        r->xy[1] = s.h_xy[2 * j + 1];
        r->tile[0] = s.h_tile[2 * j];
        r->tile[1] = s.h_tile[2 * j + 1];
        r->flags = s.h_flags[j];
        f += r->nframes;
      }
    }
    const Clock::time_point now = Clock::now();
    lk.lock();
    for (Request *r : s.reqs) {
      r->state = e == hipSuccess ? kDone : kFailed;
      r->t_done = now;
    }
    if (e == hipSuccess) {
      srv->st_batches += 1;
      srv->st_requests += (int64_t)s.reqs.size();
      srv->st_frames += s.nq;
      srv->st_max_batch = std::max<int64_t>(srv->st_max_batch, s.nq);
    } else {
      srv->err_code = HLOC_EDEVICE;
      srv->err_msg = std::string("hipEventSynchronize: ") + hipGetErrorString(e);
    }
    s.reqs.clear();
    s.busy = false;
    srv->inflight.pop_front();
    srv->cv_done.notify_all();
    srv->cv_launch.notify_one();
  }
}

void destroy(hloc_server *srv) {
  for (Slot &s : srv->slots) free_slot(s);
  for (auto &kv : srv->reqs) delete kv.second;
  delete srv;
}

}  // namespace

extern "C" {

int hloc_server_create(hloc_db *db, const hloc_server_config *cfg, hloc_server **out) {
  if (!out) return fail(HLOC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!db || !cfg) return fail(HLOC_EINVAL, "db and cfg must be non-NULL");
  const hloc_server_config c = *cfg;
  if (c.k < 1 || c.k > HLOC_MAX_K) return fail(HLOC_EINVAL, "k must be in 1..%d", HLOC_MAX_K);
  if (c.n_regions < 1) return fail(HLOC_EINVAL, "n_regions must be >= 1");
  if (c.max_batch_frames < 1) return fail(HLOC_EINVAL, "max_batch_frames must be >= 1");
  if (c.max_slots < 1) return fail(HLOC_EINVAL, "max_slots must be >= 1");
  if (c.max_queue_frames < c.max_batch_frames)
    return fail(HLOC_EINVAL, "max_queue_frames must be >= max_batch_frames");
  if (c.hbm_budget_bytes < 0) return fail(HLOC_EINVAL, "hbm_budget_bytes must be >= 0");
  Plan full;
  CHK(make_plan(db, c.max_batch_frames, c.k, c.n_regions, c.max_batch_frames, c.precision, &full));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  hloc_server *srv = new (std::nothrow) hloc_server();
  if (!srv) return fail(HLOC_ENOMEM, "host allocation failed");
  srv->db = db;
  srv->cfg = c;
  {
    hloc_ws probe;
    probe.db = db;
    size_t ws_bytes = 0;
    CHK(ensure_workspace(&probe, full, false, &ws_bytes));
    srv->slot_bytes = ws_bytes + io_bytes(db, c.max_batch_frames, c.k);
  }
  int64_t nslots = c.max_slots;
  if (c.hbm_budget_bytes > 0)
    nslots = std::min<int64_t>(nslots, c.hbm_budget_bytes / (int64_t)srv->slot_bytes);
  if (nslots < 1) {
    const size_t need = srv->slot_bytes;
    delete srv;
    return fail(HLOC_ENOMEM, "budget of %lld bytes is below one batch slot (%zu bytes)",
                (long long)c.hbm_budget_bytes, need);
  }
  srv->slots.resize((size_t)nslots);
  for (Slot &s : srv->slots) {
    const int rc = make_slot(srv, full, s);
    if (rc != HLOC_OK) {
      destroy(srv);
      return rc;
    }
  }
  srv->launcher = std::thread(launcher_main, srv);
  srv->completer = std::thread(completer_main, srv);
  ++db->servers;
  *out = srv;
  return HLOC_OK;
}

int hloc_server_submit(hloc_server *srv, const float *frames, int32_t nframes, int32_t k_req,
                       uint64_t *ticket) {
  if (!srv || !frames || !ticket) return fail(HLOC_EINVAL, "srv, frames and ticket must be non-NULL");
  if (nframes < 1 || nframes > srv->cfg.max_batch_frames)
    return fail(HLOC_EINVAL, "nframes must be in 1..%d (got %d)", srv->cfg.max_batch_frames, nframes);
  if (k_req < 1 || k_req > srv->cfg.k)
    return fail(HLOC_EINVAL, "k_req must be in 1..%d (got %d)", srv->cfg.k, k_req);
  if ((int64_t)nframes * k_req > HLOC_MAX_REQUEST_CANDIDATES)
    return fail(HLOC_EINVAL, "a request may pool at most %d candidates", HLOC_MAX_REQUEST_CANDIDATES);
  Request *r = new (std::nothrow) Request();
  if (!r) return fail(HLOC_ENOMEM, "host allocation failed");
  r->nframes = nframes;
  r->k = k_req;
  r->frames.assign(frames, frames + (size_t)nframes * srv->db->d);
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->err_code != HLOC_OK) {
    delete r;
    return fail(srv->err_code, "the server stopped after an error: %s", srv->err_msg.c_str());
  }
  if (srv->queued_frames + nframes > srv->cfg.max_queue_frames) {
    delete r;
    ++srv->st_refused;
    return fail(HLOC_EBUSY, "%lld frames are waiting (limit %d)", (long long)srv->queued_frames,
                srv->cfg.max_queue_frames);
  }
  r->ticket = srv->next_ticket++;
  r->t_submit = Clock::now();
  srv->queue.push_back(r);
  srv->reqs[r->ticket] = r;
  srv->queued_frames += nframes;
  srv->st_peak_queue = std::max(srv->st_peak_queue, srv->queued_frames);
  *ticket = r->ticket;
  srv->cv_launch.notify_one();
  return HLOC_OK;
}

int hloc_server_wait(hloc_server *srv, uint64_t ticket, int32_t timeout_ms, int64_t *idx,
                     float *dist, double *xy, int32_t *tile, int32_t *flags, double *latency_ms) {
  if (!srv) return fail(HLOC_EINVAL, "srv is NULL");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return fail(HLOC_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second;
  auto ready = [&] { return r->state == kDone || r->state == kFailed || srv->err_code != HLOC_OK; };
  if (timeout_ms < 0) {
    srv->cv_done.wait(lk, ready);
  } else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
    return fail(HLOC_ETIMEDOUT, "request %llu is not done yet", (unsigned long long)ticket);
  }
  if (r->state != kDone) {
    if (r->state == kFailed) {
      srv->reqs.erase(it);
      delete r;
    }
    return fail(HLOC_EDEVICE, "the server stopped after an error: %s", srv->err_msg.c_str());
  }
  if (idx) std::memcpy(idx, r->idx.data(), r->idx.size() * sizeof(int64_t));
  if (dist) std::memcpy(dist, r->dist.data(), r->dist.size() * sizeof(float));
  if (xy) std::memcpy(xy, r->xy, sizeof r->xy);
  if (tile) std::memcpy(tile, r->tile, sizeof r->tile);
  if (flags) *flags = r->flags;
  if (latency_ms)
    *latency_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
  srv->reqs.erase(it);
  delete r;
  return HLOC_OK;
}

int hloc_server_stats(hloc_server *srv, int64_t *out, int32_t n) {
  if (!srv || !out || n < 0) return fail(HLOC_EINVAL, "srv and out must be non-NULL, n >= 0");
  std::lock_guard<std::mutex> lk(srv->mu);
  const int64_t vals[10] = {(int64_t)srv->slots.size(), (int64_t)srv->slot_bytes, srv->st_batches,
                            srv->st_requests, srv->st_frames, srv->st_max_batch,
                            srv->queued_frames, srv->st_peak_queue, srv->st_max_inflight,
                            srv->st_refused};
  for (int32_t i = 0; i < std::min(n, 10); ++i) out[i] = vals[i];
  return HLOC_OK;
}

void hloc_server_free(hloc_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_launch.notify_all();
  srv->cv_complete.notify_all();
  srv->cv_done.notify_all();
  if (srv->launcher.joinable()) srv->launcher.join();
  if (srv->completer.joinable()) srv->completer.join();
  DeviceGuard g(srv->db->device);
  --srv->db->servers;
  destroy(srv);
}

}  // extern "C"
