// Host side of the hloc C ABI (include/hloc.h): argument checks, device
// layout of the database, workspaces (the scratch memory of one batch in
// flight) and the sequence of kernels that localizes a batch, launched
// directly or replayed from a captured hipGraph.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "hloc_host.h"

using namespace hloc;

// Scratch memory of hloc_query_batch_static_async, which allocates nothing:
// every device the library runs on holds its own copy of this array until
// the process ends. On the host the name is only a stand-in, not a device
// address: host code uses the per-device address from hipGetSymbolAddress
// (static_scratch below), never the name.
static __device__ __align__(256) unsigned char scratch[HLOC_STATIC_SCRATCH_BYTES];

namespace hloc {
thread_local PhaseEvents *g_phase = nullptr;
}

namespace {

thread_local std::string g_err;

}  // namespace

int hloc::fail(int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

namespace hloc {

void free_buf(WsBuf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

size_t alloc_size(size_t bytes) { return std::max<size_t>(bytes + bytes / 4, 256); }

int ensure(WsBuf &b, size_t bytes) {
  if (bytes <= b.cap && b.p) return HLOC_OK;
  HIPCHK(hipDeviceSynchronize());  // the old buffer may still be in use
  free_buf(b);
  const size_t want = alloc_size(bytes);
  if (hipMalloc(&b.p, want) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(HLOC_ENOMEM, "device allocation of %zu bytes failed", want);
  }
  b.cap = want;
  return HLOC_OK;
}

int ws_ensure(hloc_ws *ws, WsBuf &b, size_t bytes) {
  if (bytes <= b.cap && b.p) return HLOC_OK;
  drop_graph(ws);
  return ensure(b, bytes);
}

template <class T>
int dev_alloc(T **p, size_t count) {
  if (hipMalloc(reinterpret_cast<void **>(p), std::max<size_t>(count, 1) * sizeof(T)) !=
      hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(HLOC_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
  }
  return HLOC_OK;
}

template <class T>
void dev_free(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}


int make_plan(const hloc_db *db, int32_t nq, int32_t k, int32_t n_regions, int32_t nreq,
              int32_t precision, Plan *pl) {
  if (!db->has_regions) return fail(HLOC_ESTATE, "hloc_set_regions has not been called");
  if (precision == HLOC_BF16 || precision == HLOC_FP8) {
    const char *name = precision == HLOC_BF16 ? "bf16" : "fp8";
    if (!db->lp[precision].rows)
      return fail(HLOC_EUNSUPPORTED, "the %s screen needs a database built with its mirror", name);
    if (!lp_screen_supports(precision, db->dp))
      return fail(HLOC_EUNSUPPORTED, "the %s screen does not support padded length %d", name,
                  db->dp);
  } else if (precision != HLOC_FP32) {
    return fail(HLOC_EUNSUPPORTED, "screen precision %d is not available in this build", precision);
  }
  if (nq < 0) return fail(HLOC_EINVAL, "nq must be >= 0 (got %d)", nq);
  if (k < 1 || k > HLOC_MAX_K) return fail(HLOC_EINVAL, "k must be in 1..%d (got %d)", HLOC_MAX_K, k);
  if (n_regions < 1) return fail(HLOC_EINVAL, "n_regions must be >= 1 (got %d)", n_regions);
  Plan p{};
  p.nq = nq;
  p.k = k;
  p.nreq = nreq;
  p.precision = precision;
  p.nr = std::min(n_regions, db->R_nonempty);
  p.exhaustive = p.nr == db->R_nonempty;
  if (!p.exhaustive) {
    p.L1 = std::min(p.nr + kRegionMargin, db->R_nonempty);
    if (p.L1 > kMaxSurvivors)
      return fail(HLOC_EINVAL,
                  "n_regions %d is above %d and below the %d non-empty regions; pass "
                  "n_regions >= %d to search every region",
                  n_regions, kMaxSurvivors - kRegionMargin, db->R_nonempty, db->R_nonempty);
  }
  // survivors re-scored in FP64: k + 16 behind the fp32 screen, 3k behind bf16
  p.kp = std::min(precision == HLOC_FP32 ? k + kOversample : std::max(3 * k, k + kOversample),
                  kMaxSurvivors);  // 3k behind the bf16 and fp8 screens
  // bf16 coarse screens (bf16 queries, and fp8 queries when the database
  // keeps bf16 representatives) on a length the fused product supports
  p.coarse_keys = !p.exhaustive && precision != HLOC_FP32 && db->lp[HLOC_BF16].reps &&
                  coarse_gemm_supports(db->dp) && db->R < (1 << 28);
  if (p.coarse_keys) {
    const int32_t sp = coarse_gemm_splits(std::max(nq, 1), db->R, db->num_cu);
    p.creps = (db->R + sp - 1) / sp;
    p.creps = (p.creps + 31) / 32 * 32;           // whole tiles of 32
    p.csplits = (db->R + p.creps - 1) / p.creps;  // no empty range
  }
  p.cap2 = p.exhaustive ? db->n_blocks : db->h_desc_blocks[p.nr];
  const int32_t crow = std::min(db->tile_rows, kWideRows);  // the shorter chunks bound the items
  const int64_t maxch = (db->max_region + crow - 1) / crow;
  const int64_t b1 = (int64_t)nq * p.nr * maxch;
  const int64_t b2 = db->chunks_fine * (((int64_t)nq + kListFrames - 1) / kListFrames);
  p.items_bound = std::min(b1, b2);
  if (p.items_bound > INT32_MAX || (int64_t)nq * p.cap2 > ((int64_t)1 << 40))
    return fail(HLOC_EINVAL, "batch too large for one call (nq %d)", nq);
  const int32_t max_blocks = db->num_cu * db->tile_blocks;
  p.grid2 = screen_grid(p.items_bound, db->dp, max_blocks);
  const int64_t dense_items =
      (((int64_t)db->R + kRowsCoarse - 1) / kRowsCoarse) * (((int64_t)nq + kGroup - 1) / kGroup);
  p.grid1 = screen_grid(dense_items, db->dp, max_blocks);
  *pl = p;
  return HLOC_OK;
}

int ensure_workspace(hloc_ws *ws, const Plan &p, bool agg_internal, size_t *bytes,
                     const Carve *carve) {
  const hloc_db *db = ws->db;
  // with `bytes`: only add up what the buffers would take; with `carve`:
  // point each buffer into the caller's memory (256-byte aligned, in order)
  // and add up the bytes used, allocating nothing
  auto fit = [&](WsBuf &b, size_t need) -> int {
    if (carve) {
      b.p = static_cast<char *>(carve->base) + *bytes;
      b.cap = need;
      *bytes += (need + 255) / 256 * 256;
      return HLOC_OK;
    }
    if (bytes) {
      *bytes += alloc_size(need);
      return HLOC_OK;
    }
    return ws_ensure(ws, b, need);
  };
  const int64_t nq = std::max(p.nq, 1), nr = std::max(p.nr, 1);
  CHK(fit(ws->qp, (size_t)nq * db->dp * sizeof(float)));
  CHK(fit(ws->qn2, (size_t)nq * sizeof(float)));
  if (p.coarse_keys) {
    CHK(fit(ws->ckeys, (size_t)nq * p.csplits * kCgKeys * sizeof(uint64_t)));
    CHK(fit(ws->cslots, (size_t)nq * p.csplits * 4 * kCgKeep * sizeof(uint4)));
    CHK(fit(ws->cbounds, (size_t)nq * p.csplits * 4 * sizeof(uint64_t)));
    CHK(fit(ws->cdefer, (size_t)nq * sizeof(int32_t)));
  }
  if (!p.exhaustive) CHK(fit(ws->cand1, (size_t)nq * db->R * sizeof(uint32_t)));
  CHK(fit(ws->regions, (size_t)nq * nr * sizeof(int32_t)));
  CHK(fit(ws->rcount, (size_t)db->R * sizeof(int32_t)));
  CHK(fit(ws->rfill, (size_t)db->R * sizeof(int32_t)));
  CHK(fit(ws->vord, (size_t)db->R * sizeof(int32_t)));
  CHK(fit(ws->rq_off, (size_t)(db->R + 1) * sizeof(int32_t)));
  CHK(fit(ws->item_off, (size_t)(db->R + 1) * sizeof(int32_t)));
  CHK(fit(ws->cand_off, (size_t)nq * nr * sizeof(int32_t)));
  CHK(fit(ws->slot_row, (size_t)nq * nr * sizeof(int32_t)));
  CHK(fit(ws->slot_len, (size_t)nq * nr * sizeof(int32_t)));
  CHK(fit(ws->n_cand, (size_t)nq * sizeof(int32_t)));
  CHK(fit(ws->n_rows, (size_t)nq * sizeof(int32_t)));
  CHK(fit(ws->fstat, (size_t)nq * sizeof(int4)));
  CHK(fit(ws->misc, kMiscInts * sizeof(int32_t)));
  CHK(fit(ws->rq, (size_t)nq * nr * sizeof(int2)));
  CHK(fit(ws->items, (size_t)std::max<int64_t>(p.items_bound, 1) * sizeof(Item)));
  CHK(fit(ws->cand2, (size_t)nq * std::max<int64_t>(p.cap2, 1) * sizeof(uint32_t)));
  if (db->lp[HLOC_BF16].rows || db->lp[HLOC_FP8].rows) {
    CHK(fit(ws->q_lp, (size_t)nq * db->dp * (db->lp[HLOC_BF16].rows ? 2 : 1)));
    CHK(fit(ws->q_scale, (size_t)nq * sizeof(float)));
    CHK(fit(ws->q_err, (size_t)nq * sizeof(float)));
    CHK(fit(ws->q_lon, (size_t)nq * sizeof(float)));
  }
  if (db->lp[HLOC_FP8].rows && db->lp[HLOC_BF16].reps) {
    CHK(fit(ws->c_lp, (size_t)nq * db->dp * 2));
    CHK(fit(ws->c_scale, (size_t)nq * sizeof(float)));
    CHK(fit(ws->c_err, (size_t)nq * sizeof(float)));
    CHK(fit(ws->c_lon, (size_t)nq * sizeof(float)));
  }
  CHK(fit(ws->agg_big, (size_t)std::max(p.nreq, 1) * sizeof(int32_t)));
  if (agg_internal) {
    const int64_t nreq = std::max(p.nreq, 1);
    CHK(fit(ws->agg_xy, (size_t)nreq * 2 * sizeof(double)));
    CHK(fit(ws->agg_tile, (size_t)nreq * 2 * sizeof(int32_t)));
    CHK(fit(ws->agg_flags, (size_t)nreq * sizeof(int32_t)));
  }
  return HLOC_OK;
}

hipEvent_t take_event(hloc_ws *ws) {
  if (ws->ev_used == ws->ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    ws->ev_pool.push_back(e);
  }
  return ws->ev_pool[ws->ev_used++];
}

// Times consecutive phases of a query while profiling is on: begin(p) closes
// the open phase and routes the next kernel launches through event-timed
// dispatches (see launch_kernel); the destructor closes the last phase.
struct Phaser {
  hloc_ws *ws;
  int phase = -1;
  PhaseEvents pe;
  explicit Phaser(hloc_ws *w) : ws(w) {}
  void end() {
    if (phase >= 0 && pe.launches > 0 && pe.start && pe.stop)
      ws->prof.push_back({phase, pe.start, pe.stop});
    phase = -1;
    g_phase = nullptr;
  }
  void begin(int p) {
    end();
    if (!ws->prof_on) return;
    phase = p;
    pe = PhaseEvents{take_event(ws), take_event(ws), 0};
    g_phase = &pe;
  }
  ~Phaser() { end(); }
};

int enqueue_query(hloc_ws *ws, const Plan &p, const float *q, const int32_t *req_offsets,
                  const int32_t *req_k, int64_t *idx, float *dist, double *xy, int32_t *tile,
                  int32_t *flags, hipStream_t s, const int32_t *req_frames, int32_t n_frames,
                  int32_t label, int32_t label_frames) {
  const hloc_db *db = ws->db;
  const bool want_agg = xy || tile || flags;
  CHK(ensure_workspace(ws, p, want_agg && !(xy && tile && flags)));
  ws->last_nq = p.nq;
  ws->last_nr = p.nr;
  ws->last_kp = p.kp;
  int32_t *misc = as<int32_t>(ws->misc);
  if (p.nq == 0) {
    HIPCHK(launch_fill_i32(misc, kMiscInts, 0, s));
    return HLOC_OK;
  }
  float *qp = as<float>(ws->qp), *qn2 = as<float>(ws->qn2);
  int32_t *regions = as<int32_t>(ws->regions);
  Phaser ph(ws);
  ph.begin(HLOC_PHASE_PREP);
  // low-precision screens: the frames rounded the same way as the rows
  const int fmt = p.precision == HLOC_FP32 ? 0 : p.precision;
  const LpMirror *lpm = fmt ? &db->lp[fmt] : nullptr;
  // the coarse screen of fp8 queries runs on bf16 copies when there are any
  const bool coarse_bf16 = fmt == HLOC_FP8 && db->lp[HLOC_BF16].reps;
  const int cfmt = coarse_bf16 ? HLOC_BF16 : fmt;
  const LpMirror *cpm = cfmt ? &db->lp[cfmt] : nullptr;
  void *c_lp = coarse_bf16 ? ws->c_lp.p : ws->q_lp.p;
  float *c_scale = as<float>(coarse_bf16 ? ws->c_scale : ws->q_scale);
  float *c_err = as<float>(coarse_bf16 ? ws->c_err : ws->q_err);
  float *c_lon = as<float>(coarse_bf16 ? ws->c_lon : ws->q_lon);
  HIPCHK(launch_prep_queries(q, p.nq, db->d, db->dp, qp, qn2, misc, s));
  if (fmt)
    HIPCHK(launch_frames_to_lp(fmt, qp, p.nq, db->dp, ws->q_lp.p, as<float>(ws->q_scale),
                               as<float>(ws->q_err), as<float>(ws->q_lon), s));
  if (coarse_bf16 && !p.exhaustive)
    HIPCHK(launch_frames_to_lp(HLOC_BF16, qp, p.nq, db->dp, c_lp, c_scale, c_err, c_lon, s));
  // fp32 accumulation of rounded products: |q~||d~| <= 1.004 |q||d| for bf16,
  // <= (1 + 2^-4)^2 |q||d| for fp8 (relative rounding of at most 2^-4 per
  // value; subnormals are absolute and covered by the rounding-error terms)
  const double lo_fp32 = fmt == HLOC_FP8 ? 1.15 : 1.01;
  ph.begin(HLOC_PHASE_COARSE);
  const double coef = (db->dp + 16) * kUnit32 * 1.001;
  const bool masked = (label >= 0 || label_frames > 0) && db->rlabel;
  const bool coarse_lp = cfmt && cpm->reps;
  // The dense coarse stage: every frame's word against every representative,
  // then the words-mode select (FP64 re-score of the best, certificate).
  // With a frame list, only the listed frames (those the fused product's
  // keys could not decide; their count on the device).
  auto coarse_words = [&](const int32_t *list, const int32_t *count) -> int {
    ScreenArgs sa{};
    sa.rows = db->rep32;
    sa.row_n2 = db->rep_n2;
    sa.dp = db->dp;
    sa.qp = qp;
    sa.qn2 = qn2;
    sa.cand = as<uint32_t>(ws->cand1);
    sa.cap = db->R;
    sa.rows_per_item = kRowsCoarse;
    sa.dense = 1;
    sa.nrows = db->R;
    sa.nq = p.nq;
    sa.frame_list = list;
    sa.frame_count = count;
    // large batches: 64 representatives staged in LDS against 256 frames at a
    // time (the wide kernels' dense mode) instead of re-reading them per 16
    const bool wide_dense =
        !list && p.nq >= kWideDenseFrames && (coarse_lp || f32_wide_supports(db->dp));
    if (coarse_lp) {
      sa.rows_lp = cpm->reps;
      sa.q_lp = c_lp;
      sa.row_scale = cpm->rep_scale;
      sa.q_scale = c_scale;
      HIPCHK(wide_dense ? launch_screen_wide_lp(cfmt, sa, p.grid1, db->num_cu, s)
                        : launch_screen_lp(cfmt, sa, p.grid1, s));
    } else {
      HIPCHK(wide_dense ? launch_screen_wide_f32(sa, p.grid1, db->num_cu, s)
                        : launch_screen_f32(sa, p.grid1, s));
    }
    if (masked)
      HIPCHK(launch_mask_label(as<uint32_t>(ws->cand1), p.nq, db->R, db->rlabel, label,
                               label_frames, s));
    if (!list) ph.begin(HLOC_PHASE_COARSE_SELECT);
    SelRerankArgs ra{};
    ra.cand = as<uint32_t>(ws->cand1);
    ra.cap = db->R;
    ra.n_fixed = db->R;
    ra.L = p.L1;
    ra.m = p.nr;
    ra.src64 = db->rep64;
    ra.dp = db->dp;
    ra.qp = qp;
    ra.qn2 = qn2;
    ra.err_coef = coef;
    ra.max_norm = (double)db->h_rep_max * (1.0 + 1e-6);
    if (coarse_lp) {
      ra.q_err = c_err;
      ra.q_lon = c_lon;
      ra.lo_dmax = (double)cpm->rep_err * (1.0 + 1e-6);
      ra.lo_nmax = (double)cpm->rep_norm * (1.0 + 1e-6);
      ra.lo_coef = 2.0 * (1.0 + 1e-6);
      ra.err_coef = coef * (cfmt == HLOC_FP8 ? 1.15 : 1.01);
    }
    ra.nq = p.nq;
    ra.reg_out = regions;
    ra.stat_fallback = misc + 1;
    ra.frame_list = list;
    ra.frame_count = count;
    HIPCHK(launch_select_rerank(ra, s));
    return HLOC_OK;
  };
  if (p.coarse_keys) {
    // one bf16 product of frames and representatives whose epilogue keeps
    // short key lists; the select re-scores the best in FP64 and certifies,
    // and the frames it cannot decide from the keys take the dense stage
    CoarseGemmArgs ca{};
    ca.reps = cpm->reps;
    ca.rep_n2 = db->rep_n2;
    ca.frames = c_lp;
    ca.qn2 = qn2;
    ca.R = db->R;
    ca.nq = p.nq;
    ca.dp = db->dp;
    ca.splits = p.csplits;
    ca.reps_per_split = p.creps;
    if (masked) {
      ca.rlabel = db->rlabel;
      ca.label = label;
      ca.label_frames = label_frames;
    }
    ca.slots = as<uint4>(ws->cslots);
    ca.keys = as<uint64_t>(ws->ckeys);
    ca.bounds = as<uint64_t>(ws->cbounds);
    HIPCHK(launch_coarse_gemm(ca, s));
    ph.begin(HLOC_PHASE_COARSE_SELECT);
    SelRerankArgs ra{};
    ra.keys = ca.keys;
    ra.cap = (int64_t)p.csplits * kCgKeys;
    ra.n_fixed = p.csplits * kCgKeys;
    ra.bounds = ca.bounds;
    ra.n_bounds = p.csplits * 4;
    ra.defer_list = as<int32_t>(ws->cdefer);
    ra.defer_count = misc + 10;  // cleared by the prep kernel
    ra.L = p.L1;
    ra.m = p.nr;
    ra.src64 = db->rep64;
    ra.dp = db->dp;
    ra.qp = qp;
    ra.qn2 = qn2;
    ra.max_norm = (double)db->h_rep_max * (1.0 + 1e-6);
    ra.q_err = c_err;
    ra.q_lon = c_lon;
    ra.lo_dmax = (double)cpm->rep_err * (1.0 + 1e-6);
    ra.lo_nmax = (double)cpm->rep_norm * (1.0 + 1e-6);
    ra.lo_coef = 2.0 * (1.0 + 1e-6);
    ra.err_coef = coef * 1.01;
    ra.nq = p.nq;
    ra.reg_out = regions;
    ra.stat_fallback = misc + 1;
    HIPCHK(launch_select_rerank(ra, s));
    ph.begin(HLOC_PHASE_COARSE_DEFER);
    CHK(coarse_words(as<int32_t>(ws->cdefer), misc + 10));
  } else if (!p.exhaustive) {
    CHK(coarse_words(nullptr, nullptr));
  } else {
    HIPCHK(launch_broadcast_ids(db->nonempty_ids, p.nr, p.nq, regions, s));
  }
  ph.begin(HLOC_PHASE_SCHED);
  int32_t *cand_off = as<int32_t>(ws->cand_off), *n_cand = as<int32_t>(ws->n_cand);
  // wide regions: chunks the wide kernel of this screen takes
  const bool rs = fmt && lp_wide_rs(fmt, db->dp);
  const int32_t wide_rows = rs ? kWideRowsRs : std::min(db->tile_rows, kWideRows);
  HIPCHK(launch_sched(regions, p.nq, p.nr, db->R, db->reg_start, db->tile_rows, wide_rows,
                      rs ? kWideRunsRs : 1,
                      as<int32_t>(ws->rcount), as<int32_t>(ws->rfill), as<int32_t>(ws->vord),
                      as<int32_t>(ws->rq_off),
                      as<int32_t>(ws->item_off), cand_off, as<int32_t>(ws->slot_row),
                      as<int32_t>(ws->slot_len), n_cand,
                      as<int32_t>(ws->n_rows), misc + 0, as<int2>(ws->rq), as<Item>(ws->items),
                      s));
  ph.begin(HLOC_PHASE_SCREEN);
  ScreenArgs sb{};
  sb.rows = db->rows;
  sb.row_n2 = db->row_n2;
  sb.dp = db->dp;
  sb.qp = qp;
  sb.qn2 = qn2;
  sb.cand = as<uint32_t>(ws->cand2);
  sb.cap = p.cap2;
  sb.rows_per_item = db->tile_rows;
  sb.dense = 0;
  sb.items = as<Item>(ws->items);
  sb.n_items = misc + 0;
  sb.item_ctr = misc + kMiscItemCtr;
  sb.rq = as<int2>(ws->rq);
  sb.reg_start = db->reg_start;
  if (fmt) {
    sb.rows_lp = lpm->rows;
    sb.q_lp = ws->q_lp.p;
    sb.row_scale = lpm->scale;
    sb.q_scale = as<float>(ws->q_scale);
  }
  HIPCHK(fmt ? launch_screen_lp(fmt, sb, p.grid2, s) : launch_screen_f32(sb, p.grid2, s));
  ph.begin(HLOC_PHASE_SCREEN_WIDE);
  HIPCHK(fmt ? launch_screen_wide_lp(fmt, sb, p.grid2, db->num_cu, s)
             : launch_screen_wide_f32(sb, p.grid2, db->num_cu, s));
  ph.begin(HLOC_PHASE_SELECT);
  SelRerankArgs rb{};
  rb.cand = as<uint32_t>(ws->cand2);
  rb.cap = p.cap2;
  // the fine screen wrote one word per 16-row block: block positions -> rows
  // through the frame's region slots; in the exhaustive search the slots are
  // every non-empty region in id order, so the database's block table
  // serves every frame
  rb.blocks = 1;
  rb.nslots = p.exhaustive ? 0 : p.nr;
  rb.slot_off = cand_off;
  rb.slot_row = as<int32_t>(ws->slot_row);
  rb.slot_len = as<int32_t>(ws->slot_len);
  rb.blk_rows = db->blk_rows;
  rb.n_cand = n_cand;
  rb.L = (p.kp + kBlockRows - 1) / kBlockRows;  // survivor blocks: at least k' rows
  rb.m = p.k;
  rb.src32 = db->rows;
  rb.dp = db->dp;
  rb.tie_of = db->perm;
  rb.qp = qp;
  rb.qn2 = qn2;
  rb.err_coef = coef;
  rb.max_norm = (double)db->h_row_max * (1.0 + 1e-6);
  if (fmt) {
    // the roundings enter the screen through q~.d~ - q.d =
    // q~.(d~-d) + (q~-q).d~ - (q~-q).(d~-d), doubled by the -2 q.d term
    rb.q_err = as<float>(ws->q_err);
    rb.q_lon = as<float>(ws->q_lon);
    rb.lo_dmax = (double)lpm->err * (1.0 + 1e-6);
    rb.lo_nmax = (double)lpm->norm * (1.0 + 1e-6);
    rb.lo_coef = 2.0 * (1.0 + 1e-6);
    rb.err_coef = coef * lo_fp32;
  }
  rb.nq = p.nq;
  rb.idx_out = idx;
  rb.dist_out = dist;
  rb.frame_stat = as<int4>(ws->fstat);
  HIPCHK(launch_select_rerank(rb, s));
  ph.end();
  if (want_agg && p.nreq > 0) {
    AggArgs ag{};
    ag.idx = idx;
    ag.k = p.k;
    ag.nq = p.nq;
    ag.req_offsets = req_offsets;
    ag.req_k = req_k;
    ag.nreq = p.nreq;
    ag.tile_of = db->tiles;
    ag.cell = db->cell;
    ag.top_c = db->top_c;
    ag.rho = db->rho;
    ag.toler_pct = db->pct;
    ag.xy = xy ? xy : as<double>(ws->agg_xy);
    ag.tile = tile ? tile : as<int32_t>(ws->agg_tile);
    ag.flags = flags ? flags : as<int32_t>(ws->agg_flags);
    ag.big_list = as<int32_t>(ws->agg_big);
    ag.big_count = misc + 8;
    ag.num_cu = db->num_cu;
    ph.begin(HLOC_PHASE_AGGREGATE);
    HIPCHK(launch_aggregate_frames(ag, req_frames, n_frames, s));
  }
  return HLOC_OK;
}

int check_query_args(const hloc_db *db, const float *q, int32_t nq, const int32_t *req_offsets,
                     int32_t nreq, int32_t precision, const int64_t *idx, const float *dist) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (precision != HLOC_FP32 && precision != HLOC_BF16 && precision != HLOC_FP8)
    return fail(HLOC_EINVAL, "unknown precision %d", precision);
  if (nq > 0 && (!q || !idx || !dist)) return fail(HLOC_EINVAL, "q, idx and dist must be non-NULL");
  if (nreq < 0) return fail(HLOC_EINVAL, "nreq must be >= 0");
  if (!req_offsets && nreq != nq)
    return fail(HLOC_EINVAL, "without req_offsets nreq must equal nq (%d vs %d)", nreq, nq);
  return HLOC_OK;
}

int check_host_offsets(const int32_t *req_offsets, int32_t nq, int32_t nreq, int32_t k) {
  if (req_offsets) {
    if (req_offsets[0] != 0 || req_offsets[nreq] != nq)
      return fail(HLOC_EINVAL, "req_offsets must run from 0 to nq");
    for (int32_t i = 0; i < nreq; ++i) {
      if (req_offsets[i + 1] < req_offsets[i])
        return fail(HLOC_EINVAL, "req_offsets decreases at %d", i);
      if ((int64_t)(req_offsets[i + 1] - req_offsets[i]) * k > HLOC_MAX_REQUEST_CANDIDATES)
        return fail(HLOC_EINVAL, "request %d has more than %d candidates", i,
                    HLOC_MAX_REQUEST_CANDIDATES);
    }
  } else if ((int64_t)k > HLOC_MAX_REQUEST_CANDIDATES) {
    return fail(HLOC_EINVAL, "k is above the request candidate limit");
  }
  return HLOC_OK;
}

void drop_graph(hloc_ws *ws) {
  if (ws->exec) (void)hipGraphExecDestroy(ws->exec);
  if (ws->graph) (void)hipGraphDestroy(ws->graph);
  ws->exec = nullptr;
  ws->graph = nullptr;
}

// Every buffer of a workspace.
template <class F>
void for_each_buf(hloc_ws *ws, F f) {
  WsBuf *bufs[] = {&ws->vord,     &ws->qp,       &ws->qn2,      &ws->cand1,    &ws->regions, &ws->rcount,
                   &ws->rfill,    &ws->rq_off,   &ws->item_off, &ws->cand_off, &ws->n_cand,
                   &ws->misc,     &ws->rq,       &ws->items,    &ws->cand2,   &ws->agg_xy,
                   &ws->agg_tile, &ws->agg_flags, &ws->s_q,     &ws->s_off,   &ws->s_idx,
                   &ws->s_dist,   &ws->s_xy,     &ws->s_tile,   &ws->s_flags, &ws->q_lp,
                   &ws->q_scale,  &ws->q_err,    &ws->q_lon,   &ws->slot_row, &ws->slot_len, &ws->n_rows, &ws->fstat,
                   &ws->c_lp,     &ws->c_scale,  &ws->c_err,   &ws->c_lon,   &ws->agg_big,
                   &ws->lab_off,  &ws->lab_list, &ws->lab_q,  &ws->ckeys,
                   &ws->cslots,   &ws->cbounds,  &ws->cdefer};
  for (WsBuf *b : bufs) f(*b);
}

void free_ws(hloc_ws *ws) {
  if (!ws) return;
  drop_graph(ws);
  for_each_buf(ws, [](WsBuf &b) { free_buf(b); });
  for (hipEvent_t e : ws->ev_pool) (void)hipEventDestroy(e);
  if (ws->stream) (void)hipStreamDestroy(ws->stream);
  delete ws;
}

int new_ws(hloc_db *db, hloc_ws **out) {
  hloc_ws *ws = new (std::nothrow) hloc_ws();
  if (!ws) return fail(HLOC_ENOMEM, "host allocation failed");
  ws->db = db;
  if (hipStreamCreateWithFlags(&ws->stream, hipStreamNonBlocking) != hipSuccess) {
    delete ws;
    return fail(HLOC_EDEVICE, "hipStreamCreateWithFlags failed");
  }
  *out = ws;
  return HLOC_OK;
}

// Sum over regions of ceil(size / rows).
int64_t count_chunks(const hloc_db *db, int32_t rows) {
  int64_t c = 0;
  for (size_t r = 0; r + 1 < db->h_reg_start.size(); ++r)
    c += (db->h_reg_start[r + 1] - db->h_reg_start[r] + rows - 1) / rows;
  return c;
}

// Releases a low-precision mirror: the representatives' copy, and with
// rows_too the rows' copy as well.
void free_lp(LpMirror &m, bool rows_too) {
  if (m.reps) (void)hipFree(m.reps);
  if (m.rep_scale) (void)hipFree(m.rep_scale);
  m.reps = nullptr;
  m.rep_scale = nullptr;
  if (rows_too) {
    if (m.rows) (void)hipFree(m.rows);
    if (m.scale) (void)hipFree(m.scale);
    m.rows = nullptr;
    m.scale = nullptr;
  }
}

void free_db_data(hloc_db *db) {
  free_ws(db->ws0);
  db->ws0 = nullptr;
  dev_free(db->rows);
  for (LpMirror &m : db->lp) free_lp(m, true);
  dev_free(db->row_n2);
  dev_free(db->perm);
  dev_free(db->xy);
  dev_free(db->tiles);
  dev_free(db->norm_max);
  dev_free(db->reg_start);
  dev_free(db->nonempty_ids);
  dev_free(db->rlabel);
  dev_free(db->rep64);
  dev_free(db->rep32);
  dev_free(db->rep_n2);
  dev_free(db->blk_rows);
  if (db->stream) (void)hipStreamDestroy(db->stream);
  db->stream = nullptr;
}

int compute_tiles(hloc_db *db) {
  HIPCHK(launch_tiles(db->xy, db->n, db->cell, db->tiles, db->stream));
  HIPCHK(hipStreamSynchronize(db->stream));
  return HLOC_OK;
}

int query_async(hloc_ws *ws, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                const int32_t *req_offsets, int32_t nreq, int32_t precision, int64_t *idx,
                float *dist, double *xy, int32_t *tile, int32_t *flags, hipStream_t s) {
  hloc_db *db = ws->db;
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  Plan p;
  CHK(make_plan(db, nq, k, n_regions, nreq, precision, &p));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  return enqueue_query(ws, p, q, req_offsets, nullptr, idx, dist, xy, tile, flags, s);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the static scratch array on device `dev` (current),
// looked up once per device.
int static_scratch(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(HLOC_EDEVICE, "device %d is beyond the %d devices of the scratch table", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return fail(HLOC_EDEVICE, "address of the static scratch array: %s", hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HLOC_OK;
}

int info_of(hloc_ws *ws, int64_t *out, int32_t n) {
  DeviceGuard g(ws->db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  int32_t misc[16] = {0};
  if (ws->misc.p) HIPCHK(hipMemcpy(misc, ws->misc.p, sizeof misc, hipMemcpyDeviceToHost));
  int64_t total = 0, fine_fb = 0, max_n = 0, chunked = 0, band = 0, rows = 0;
  if (ws->last_nq > 0 && ws->n_rows.p) {
    std::vector<int32_t> nc(ws->last_nq);
    HIPCHK(hipMemcpy(nc.data(), ws->n_rows.p, nc.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int32_t v : nc) total += v;
  }
  if (ws->last_nq > 0 && ws->fstat.p) {
    // the fine select's per-frame records of the last batch
    std::vector<int4> fs(ws->last_nq);
    HIPCHK(hipMemcpy(fs.data(), ws->fstat.p, fs.size() * sizeof(int4), hipMemcpyDeviceToHost));
    for (const int4 &r : fs) {
      max_n = std::max<int64_t>(max_n, r.x);
      rows += r.y;
      band += r.z;
      fine_fb += r.w & 1;
      chunked += (r.w >> 1) & 1;
    }
  }
  const int64_t vals[11] = {misc[0], misc[1], fine_fb, max_n,   ws->last_kp, total,
                            misc[4], chunked, band,    rows,    misc[10]};
  for (int32_t i = 0; i < std::min(n, 11); ++i) out[i] = vals[i];
  return HLOC_OK;
}

}  // namespace hloc

extern "C" {

const char *hloc_last_error(void) { return g_err.c_str(); }

int hloc_build_db(const float *feats, int64_t n, int32_t d, const double *xy, uint32_t mirrors,
                  hloc_db **out) {
  if (!out) return fail(HLOC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!feats || !xy) return fail(HLOC_EINVAL, "feats and xy must be non-NULL");
  if (n < 1 || n > INT32_MAX) return fail(HLOC_EINVAL, "n must be in 1..2^31-1 (got %lld)", (long long)n);
  if (d < 1 || d > HLOC_MAX_DIM) return fail(HLOC_EINVAL, "d must be in 1..%d (got %d)", HLOC_MAX_DIM, d);
  if (mirrors & ~(uint32_t)(HLOC_MIRROR_BF16 | HLOC_MIRROR_FP8))
    return fail(HLOC_EUNSUPPORTED, "mirror flags 0x%x are not available in this build", mirrors);
  const int64_t nd = n * (int64_t)d;
  for (int64_t i = 0; i < nd; ++i)
    if (!std::isfinite(feats[i]))
      return fail(HLOC_EINVAL, "feature value %lld (row %lld) is not finite", (long long)i,
                  (long long)(i / d));
  double max_abs = 0.0;
  for (int64_t i = 0; i < 2 * n; ++i) {
    if (!std::isfinite(xy[i]))
      return fail(HLOC_EINVAL, "position value %lld is not finite", (long long)i);
    max_abs = std::max(max_abs, std::fabs(xy[i]));
  }
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hloc_db *db = new (std::nothrow) hloc_db();
  if (!db) return fail(HLOC_ENOMEM, "host allocation failed");
  db->device = dev;
  db->n = n;
  db->d = d;
  db->dp = (d + 31) / 32 * 32;
  db->max_abs_coord = max_abs;
  db->mirrors = mirrors;
  auto bail = [&](int rc) {
    free_db_data(db);
    delete db;
    return rc;
  };
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return bail(fail(HLOC_EDEVICE, "hipGetDeviceProperties failed"));
  db->num_cu = std::max(1, prop.multiProcessorCount);
  if (hipStreamCreateWithFlags(&db->stream, hipStreamNonBlocking) != hipSuccess)
    return bail(fail(HLOC_EDEVICE, "hipStreamCreateWithFlags failed"));
  int rc;
  if ((rc = new_ws(db, &db->ws0))) return bail(rc);
  hipError_t pe = prepare_kernels();
  if (pe != hipSuccess) return bail(fail(HLOC_EDEVICE, "kernel set-up failed: %s", hipGetErrorString(pe)));
  if ((rc = dev_alloc(&db->rows, (size_t)n * db->dp)) || (rc = dev_alloc(&db->row_n2, (size_t)n)) ||
      (rc = dev_alloc(&db->perm, (size_t)n)) || (rc = dev_alloc(&db->xy, (size_t)n * 2)) ||
      (rc = dev_alloc(&db->tiles, (size_t)n)) || (rc = dev_alloc(&db->norm_max, kNormSlots)))
    return bail(rc);
  float *tmp = nullptr;
  if ((rc = dev_alloc(&tmp, (size_t)nd))) return bail(rc);
  db->h_perm.resize(n);
  std::iota(db->h_perm.begin(), db->h_perm.end(), 0);
  hipError_t e = hipMemcpy(tmp, feats, (size_t)nd * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db->perm, db->h_perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(db->xy, xy, (size_t)n * 2 * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemsetAsync(db->norm_max, 0, kNormSlots * sizeof(float), db->stream);
  if (e == hipSuccess) e = launch_gather_rows(tmp, db->perm, n, d, d, db->rows, db->dp, db->stream);
  if (e == hipSuccess) e = launch_row_norms(db->rows, n, db->dp, db->row_n2, db->norm_max, db->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(db->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) return bail(fail(HLOC_EDEVICE, "database upload failed: %s", hipGetErrorString(e)));
  if ((rc = compute_tiles(db))) return bail(rc);
  *out = db;
  return HLOC_OK;
}

int hloc_set_regions(hloc_db *db, const int32_t *region_of, int32_t n_regions_total,
                     const float *reps) {
  if (!db || !region_of) return fail(HLOC_EINVAL, "db and region_of must be non-NULL");
  if (db->servers > 0) return fail(HLOC_ESTATE, "a request server is using the database");
  if (n_regions_total < 1) return fail(HLOC_EINVAL, "n_regions_total must be >= 1");
  const int64_t n = db->n;
  const int32_t R = n_regions_total;
  std::vector<int64_t> sizes(R, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int32_t r = region_of[i];
    if (r < 0 || r >= R)
      return fail(HLOC_EINVAL, "region_of[%lld] = %d is outside [0, %d)", (long long)i, r, R);
    ++sizes[r];
  }
  if (reps) {
    for (int64_t i = 0; i < (int64_t)R * db->d; ++i)
      if (!std::isfinite(reps[i])) return fail(HLOC_EINVAL, "representative value %lld is not finite", (long long)i);
  }
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  // counting sort of the rows by region, stable in the original index
  std::vector<int64_t> start(R + 1, 0);
  for (int32_t r = 0; r < R; ++r) start[r + 1] = start[r] + sizes[r];
  std::vector<int32_t> new_perm(n), src_row(n), inv_cur(n);
  {
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < n; ++i) new_perm[fill[region_of[i]]++] = (int32_t)i;
  }
  for (int64_t i = 0; i < n; ++i) inv_cur[db->h_perm[i]] = (int32_t)i;
  for (int64_t i = 0; i < n; ++i) src_row[i] = inv_cur[new_perm[i]];
  // release the old region data (and the labels of the old regions); graphs
  // captured before hold their addresses
  ++db->gen;
  dev_free(db->rlabel);
  db->n_labels = 0;
  db->h_label_nonempty.clear();
  dev_free(db->reg_start);
  dev_free(db->nonempty_ids);
  dev_free(db->rep64);
  dev_free(db->rep32);
  dev_free(db->rep_n2);
  dev_free(db->blk_rows);
  for (LpMirror &m : db->lp) free_lp(m, true);
  db->has_regions = false;
  int rc;
  float *new_rows = nullptr;
  int32_t *d_src = nullptr;
  if ((rc = dev_alloc(&new_rows, (size_t)n * db->dp))) return rc;
  if ((rc = dev_alloc(&d_src, (size_t)n))) {
    dev_free(new_rows);
    return rc;
  }
  hipError_t e = hipMemcpy(d_src, src_row.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_gather_rows(db->rows, d_src, n, db->dp, db->dp, new_rows, db->dp, db->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(db->stream);
  dev_free(d_src);
  if (e != hipSuccess) {
    dev_free(new_rows);
    return fail(HLOC_EDEVICE, "row re-layout failed: %s", hipGetErrorString(e));
  }
  dev_free(db->rows);
  db->rows = new_rows;
  db->h_perm = new_perm;
  std::vector<int32_t> ids;
  for (int32_t r = 0; r < R; ++r)
    if (sizes[r] > 0) ids.push_back(r);
  // 16-row blocks of every region in id order (the exhaustive search's
  // candidate list)
  std::vector<int2> blk;
  blk.reserve((size_t)(n / kBlockRows + R));
  for (int32_t r = 0; r < R; ++r)
    for (int64_t b = start[r]; b < start[r + 1]; b += kBlockRows)
      blk.push_back(make_int2((int)b, (int)std::min<int64_t>(kBlockRows, start[r + 1] - b)));
  if ((rc = dev_alloc(&db->reg_start, (size_t)R + 1)) || (rc = dev_alloc(&db->nonempty_ids, ids.size())) ||
      (rc = dev_alloc(&db->rep64, (size_t)R * db->dp)) || (rc = dev_alloc(&db->rep32, (size_t)R * db->dp)) ||
      (rc = dev_alloc(&db->rep_n2, (size_t)R)) || (rc = dev_alloc(&db->blk_rows, blk.size())))
    return rc;
  HIPCHK(hipMemcpy(db->blk_rows, blk.data(), blk.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(db->perm, new_perm.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(db->reg_start, start.data(), (size_t)(R + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(db->nonempty_ids, ids.data(), ids.size() * sizeof(int32_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemsetAsync(db->norm_max, 0, kNormSlots * sizeof(float), db->stream));
  HIPCHK(launch_row_norms(db->rows, n, db->dp, db->row_n2, db->norm_max, db->stream));
  for (int fmt : {HLOC_BF16, HLOC_FP8}) {
    if (!(db->mirrors & (fmt == HLOC_BF16 ? HLOC_MIRROR_BF16 : HLOC_MIRROR_FP8))) continue;
    LpMirror &m = db->lp[fmt];
    float *mx = db->norm_max + 4 * fmt - 2;
    if ((rc = dev_alloc(reinterpret_cast<uint8_t **>(&m.rows), (size_t)n * db->dp * lp_bytes(fmt))))
      return rc;
    if (fmt == HLOC_FP8 && (rc = dev_alloc(&m.scale, (size_t)n))) return rc;
    HIPCHK(launch_rows_to_lp(fmt, db->rows, n, db->dp, m.rows, m.scale, mx, mx + 1, db->stream));
  }
  if (reps) {
    std::vector<double> r64((size_t)R * db->dp, 0.0);
    for (int32_t r = 0; r < R; ++r)
      for (int32_t c = 0; c < db->d; ++c) r64[(size_t)r * db->dp + c] = reps[(size_t)r * db->d + c];
    HIPCHK(hipMemcpy(db->rep64, r64.data(), r64.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    HIPCHK(launch_region_means(db->rows, db->reg_start, R, db->dp, db->rep64, db->stream));
  }
  HIPCHK(launch_rep_finish(db->rep64, db->reg_start, R, db->dp, db->rep32, db->rep_n2,
                           db->norm_max + 1, db->stream));
  // representatives: in each mirrored format; bf16 ones also beside an fp8
  // mirror, for the coarse screen of fp8 queries (a bound 32 times tighter
  // than fp8's, at 4 MB for 4,096 x 512)
  for (int fmt : {HLOC_BF16, HLOC_FP8}) {
    LpMirror &m = db->lp[fmt];
    if (!m.rows && !(fmt == HLOC_BF16 && db->lp[HLOC_FP8].rows)) continue;
    float *mx = db->norm_max + 4 * fmt - 2;
    if ((rc = dev_alloc(reinterpret_cast<uint8_t **>(&m.reps), (size_t)R * db->dp * lp_bytes(fmt))))
      return rc;
    if (fmt == HLOC_FP8 && (rc = dev_alloc(&m.rep_scale, (size_t)R))) return rc;
    HIPCHK(launch_rows_to_lp(fmt, db->rep32, R, db->dp, m.reps, m.rep_scale, mx + 2, mx + 3,
                             db->stream));
  }
  float mx[kNormSlots];
  HIPCHK(hipMemcpyAsync(mx, db->norm_max, sizeof mx, hipMemcpyDeviceToHost, db->stream));
  HIPCHK(hipStreamSynchronize(db->stream));
  db->h_row_max = mx[0];
  db->h_rep_max = mx[1];
  for (int fmt : {HLOC_BF16, HLOC_FP8}) {
    const float *v = mx + 4 * fmt - 2;
    db->lp[fmt].err = v[0];
    db->lp[fmt].norm = v[1];
    db->lp[fmt].rep_err = v[2];
    db->lp[fmt].rep_norm = v[3];
  }
  db->R = R;
  db->R_nonempty = (int32_t)ids.size();
  db->h_reg_start = start;
  std::vector<int64_t> desc(sizes);
  std::sort(desc.begin(), desc.end(), std::greater<int64_t>());
  db->h_desc_prefix.assign(R + 1, 0);
  db->h_desc_blocks.assign(R + 1, 0);
  for (int32_t r = 0; r < R; ++r) {
    db->h_desc_prefix[r + 1] = db->h_desc_prefix[r] + desc[r];
    // block counts order like the sizes
    db->h_desc_blocks[r + 1] = db->h_desc_blocks[r] + (desc[r] + kBlockRows - 1) / kBlockRows;
  }
  db->n_blocks = (int64_t)blk.size();
  db->max_region = desc.empty() ? 0 : desc[0];
  db->chunks_fine = count_chunks(db, std::min(db->tile_rows, kWideRows));
  db->has_regions = true;
  return HLOC_OK;
}

int hloc_set_aggregation(hloc_db *db, double cell_m, int32_t top_c, double radius_m,
                         int32_t toler_pct) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (db->servers > 0) return fail(HLOC_ESTATE, "a request server is using the database");
  if (!(cell_m > 0.0) || !std::isfinite(cell_m)) return fail(HLOC_EINVAL, "cell_m must be > 0");
  if (top_c < 1 || top_c > HLOC_MAX_TOP_C) return fail(HLOC_EINVAL, "top_c must be in 1..%d", HLOC_MAX_TOP_C);
  if (!(radius_m >= 0.0) || !std::isfinite(radius_m)) return fail(HLOC_EINVAL, "radius_m must be >= 0");
  if (toler_pct < 0 || toler_pct > 100) return fail(HLOC_EINVAL, "toler_pct must be in 0..100");
  if (db->max_abs_coord / cell_m >= 1073741824.0)
    return fail(HLOC_EINVAL, "a position lies 2^30 or more tiles from the origin at cell %g m", cell_m);
  const double rr = std::floor(radius_m / cell_m + 0.5);
  if (rr > 1073741824.0) return fail(HLOC_EINVAL, "radius_m / cell_m is too large");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  ++db->gen;  // captured graphs hold the old constants
  db->cell = cell_m;
  db->top_c = top_c;
  db->radius = radius_m;
  db->rho = (int32_t)rr;
  db->pct = toler_pct;
  return compute_tiles(db);
}

int hloc_ws_create(hloc_db *db, hloc_ws **out) {
  if (!out) return fail(HLOC_EINVAL, "out is NULL");
  *out = nullptr;
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  CHK(new_ws(db, out));
  ++db->user_ws;
  return HLOC_OK;
}

void hloc_ws_free(hloc_ws *ws) {
  if (!ws) return;
  DeviceGuard g(ws->db->device);
  (void)hipDeviceSynchronize();
  --ws->db->user_ws;
  free_ws(ws);
}

int hloc_ws_reserve(hloc_ws *ws, int32_t nq_max, int32_t nreq_max, int32_t k_max,
                    int32_t n_regions_max) {
  if (!ws) return fail(HLOC_EINVAL, "ws is NULL");
  if (nreq_max < 0) return fail(HLOC_EINVAL, "nreq_max must be >= 0");
  Plan p;
  CHK(make_plan(ws->db, nq_max, k_max, n_regions_max, nreq_max, HLOC_FP32, &p));
  DeviceGuard g(ws->db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  return ensure_workspace(ws, p, true);
}

int hloc_reserve(hloc_db *db, int32_t nq_max, int32_t nreq_max, int32_t k_max,
                 int32_t n_regions_max) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  return hloc_ws_reserve(db->ws0, nq_max, nreq_max, k_max, n_regions_max);
}

int hloc_ws_query_async(hloc_ws *ws, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                        const int32_t *req_offsets, int32_t nreq, int32_t precision,
                        int64_t *idx, float *dist, double *xy, int32_t *tile, int32_t *flags,
                        void *stream) {
  if (!ws) return fail(HLOC_EINVAL, "ws is NULL");
  return query_async(ws, q, nq, k, n_regions, req_offsets, nreq, precision, idx, dist, xy, tile,
                     flags, reinterpret_cast<hipStream_t>(stream));
}

int hloc_query_windows_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                             int32_t n_regions, const int32_t *req_offsets,
                             const int32_t *req_frames, int32_t n_list, int32_t nreq,
                             int32_t precision, int64_t *idx, float *dist, double *xy,
                             int32_t *tile, int32_t *flags, void *stream) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (nreq > 0 && (!req_offsets || !req_frames))
    return fail(HLOC_EINVAL, "req_offsets and req_frames must be non-NULL");
  if (n_list < 0) return fail(HLOC_EINVAL, "n_list must be >= 0 (got %d)", n_list);
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  Plan p;
  CHK(make_plan(db, nq, k, n_regions, nreq, precision, &p));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  return enqueue_query(db->ws0, p, q, req_offsets, nullptr, idx, dist, xy, tile, flags,
                       reinterpret_cast<hipStream_t>(stream), req_frames, n_list);
}

int hloc_set_region_labels(hloc_db *db, const int32_t *labels, int32_t n_labels) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (!db->has_regions) return fail(HLOC_ESTATE, "hloc_set_regions has not been called");
  if (db->servers > 0) return fail(HLOC_ESTATE, "a request server is using this database");
  if (!labels) return fail(HLOC_EINVAL, "labels is NULL");
  if (n_labels < 1 || n_labels > HLOC_MAX_LABELS)
    return fail(HLOC_EINVAL, "n_labels must be in 1..%d (got %d)", HLOC_MAX_LABELS, n_labels);
  std::vector<int32_t> nonempty((size_t)n_labels, 0);
  for (int32_t r = 0; r < db->R; ++r) {
    if (labels[r] < 0 || labels[r] >= n_labels)
      return fail(HLOC_EINVAL, "labels[%d] = %d is outside [0, %d)", r, labels[r], n_labels);
    if (db->h_reg_start[r + 1] > db->h_reg_start[r]) ++nonempty[(size_t)labels[r]];
  }
  for (int32_t p = 0; p < n_labels; ++p)
    if (nonempty[(size_t)p] == 0)
      return fail(HLOC_EINVAL, "label %d has no non-empty region", p);
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());  // a batch in flight may read the old labels
  ++db->gen;
  dev_free(db->rlabel);
  db->n_labels = 0;
  // empty regions get label -1: a label's pass masks them with the other
  // labels' regions (its survivors may outnumber its non-empty regions, and
  // an empty region's zero representative must not be re-scored as a region)
  std::vector<int32_t> dev_labels(labels, labels + db->R);
  for (int32_t r = 0; r < db->R; ++r)
    if (db->h_reg_start[r + 1] == db->h_reg_start[r]) dev_labels[(size_t)r] = -1;
  CHK(dev_alloc(&db->rlabel, (size_t)db->R));
  HIPCHK(hipMemcpy(db->rlabel, dev_labels.data(), (size_t)db->R * sizeof(int32_t),
                   hipMemcpyHostToDevice));
  db->h_label_nonempty = nonempty;
  db->n_labels = n_labels;
  return HLOC_OK;
}

int hloc_query_labels_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                            int32_t n_regions, int32_t n_labels, const int32_t *req_offsets,
                            int32_t nreq, int32_t precision, int64_t *idx, float *dist,
                            double *xy, int32_t *tile, int32_t *flags, void *stream) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  if (db->n_labels < 1) return fail(HLOC_ESTATE, "hloc_set_region_labels has not been called");
  if (n_labels != db->n_labels)
    return fail(HLOC_EINVAL, "n_labels %d differs from the %d labels set on the database",
                n_labels, db->n_labels);
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  if (nreq > 0 && (!xy || !tile || !flags))
    return fail(HLOC_EINVAL, "xy, tile and flags must be non-NULL");
  if (n_regions < 1) return fail(HLOC_EINVAL, "n_regions must be >= 1 (got %d)", n_regions);
  if (nq == 0 && nreq > 0) return fail(HLOC_EINVAL, "requests need frames (nq is 0)");
  const int32_t P = db->n_labels;
  if ((int64_t)nq * P > INT32_MAX) return fail(HLOC_EINVAL, "nq x labels too large");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hloc_ws *ws = db->ws0;
  const int32_t min_ne =
      *std::min_element(db->h_label_nonempty.begin(), db->h_label_nonempty.end());
  if (P > 1 && n_regions <= min_ne && nq > 0) {
    // every label has n_regions regions: one batch holding the frames once
    // per label (frame p * nq + f is frame f under label p) writes the
    // label-major slabs of idx and dist in one pass
    Plan pl;
    CHK(make_plan(db, nq * P, k, n_regions, nreq, precision, &pl));
    const size_t fbytes = (size_t)nq * db->d * sizeof(float);
    CHK(ws_ensure(ws, ws->lab_q, fbytes * (size_t)P));
    for (int32_t p = 0; p < P; ++p)
      HIPCHK(hipMemcpyAsync(static_cast<char *>(ws->lab_q.p) + fbytes * (size_t)p, q, fbytes,
                            hipMemcpyDeviceToDevice, s));
    CHK(enqueue_query(ws, pl, as<float>(ws->lab_q), nullptr, nullptr, idx, dist, nullptr,
                      nullptr, nullptr, s, nullptr, 0, -1, nq));
  } else {
    // one search per label, each writing its nq x k slab of idx and dist
    for (int32_t p = 0; p < P; ++p) {
      Plan pl;
      CHK(make_plan(db, nq, k, std::min(n_regions, db->h_label_nonempty[(size_t)p]), nreq,
                    precision, &pl));
      CHK(enqueue_query(ws, pl, q, nullptr, nullptr, idx + (int64_t)p * nq * k,
                        dist + (int64_t)p * nq * k, nullptr, nullptr, nullptr, s, nullptr, 0,
                        P > 1 ? p : -1));
    }
  }
  if (nreq == 0) return HLOC_OK;
  // every request pools its frames' lists under every label
  CHK(ws_ensure(ws, ws->lab_off, (size_t)(nreq + 1) * sizeof(int32_t)));
  CHK(ws_ensure(ws, ws->lab_list, (size_t)std::max<int64_t>((int64_t)nq * P, 1) * sizeof(int32_t)));
  int32_t *lab_off = as<int32_t>(ws->lab_off), *lab_list = as<int32_t>(ws->lab_list);
  HIPCHK(launch_label_lists(req_offsets, nreq, nq, P, lab_off, lab_list, s));
  AggArgs ag{};
  ag.idx = idx;
  ag.k = k;
  ag.nq = nq * P;
  ag.req_offsets = lab_off;
  ag.req_k = nullptr;
  ag.nreq = nreq;
  ag.tile_of = db->tiles;
  ag.cell = db->cell;
  ag.top_c = db->top_c;
  ag.rho = db->rho;
  ag.toler_pct = db->pct;
  ag.xy = xy;
  ag.tile = tile;
  ag.flags = flags;
  ag.big_list = as<int32_t>(ws->agg_big);
  ag.big_count = as<int32_t>(ws->misc) + 8;  // cleared by the last search's prep
  ag.num_cu = db->num_cu;
  HIPCHK(launch_aggregate_frames(ag, lab_list, nq * P, s));
  return HLOC_OK;
}

int hloc_query_batch_async(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                           const int32_t *req_offsets, int32_t nreq, int32_t precision,
                           int64_t *idx, float *dist, double *xy, int32_t *tile, int32_t *flags,
                           void *stream) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  return query_async(db->ws0, q, nq, k, n_regions, req_offsets, nreq, precision, idx, dist, xy,
                     tile, flags, reinterpret_cast<hipStream_t>(stream));
}

int hloc_query_batch_static_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                                  int32_t n_regions, const int32_t *req_offsets, int32_t nreq,
                                  int32_t precision, int64_t *idx, float *dist, double *xy,
                                  int32_t *tile, int32_t *flags, void *stream) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  Plan p;
  CHK(make_plan(db, nq, k, n_regions, nreq, precision, &p));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  void *base = nullptr;
  CHK(static_scratch(db->device, &base));
  // a workspace record on the stack whose buffers all point into the array:
  // the sizing inside enqueue_query then finds every buffer large enough
  hloc_ws ws;
  ws.db = db;
  const bool agg_internal = (xy || tile || flags) && !(xy && tile && flags);
  size_t used = 0;
  const Carve carve{base};
  CHK(ensure_workspace(&ws, p, agg_internal, &used, &carve));
  if (used > (size_t)HLOC_STATIC_SCRATCH_BYTES)
    return fail(HLOC_EINVAL,
                "the batch needs %zu bytes of scratch memory, above the %zu bytes of the static "
                "array (send fewer frames)",
                used, (size_t)HLOC_STATIC_SCRATCH_BYTES);
  return enqueue_query(&ws, p, q, req_offsets, nullptr, idx, dist, xy, tile, flags,
                       reinterpret_cast<hipStream_t>(stream));
}

int hloc_ws_capture(hloc_ws *ws, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                    const int32_t *req_offsets, int32_t nreq, int32_t precision, int64_t *idx,
                    float *dist, double *xy, int32_t *tile, int32_t *flags) {
  if (!ws) return fail(HLOC_EINVAL, "ws is NULL");
  hloc_db *db = ws->db;
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  Plan p;
  CHK(make_plan(db, nq, k, n_regions, nreq, precision, &p));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  CHK(ensure_workspace(ws, p, true));  // no allocation may happen while capturing
  HIPCHK(hipStreamSynchronize(ws->stream));
  drop_graph(ws);
  const bool prof = ws->prof_on;
  ws->prof_on = false;
  HIPCHK(hipStreamBeginCapture(ws->stream, hipStreamCaptureModeThreadLocal));
  const int rc = enqueue_query(ws, p, q, req_offsets, nullptr, idx, dist, xy, tile, flags,
                               ws->stream);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(ws->stream, &graph);
  ws->prof_on = prof;
  if (rc != HLOC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (ec != hipSuccess) return fail(HLOC_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(ec));
  const hipError_t ei = hipGraphInstantiate(&ws->exec, graph, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(graph);
    ws->exec = nullptr;
    return fail(HLOC_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  ws->graph = graph;
  ws->graph_gen = db->gen;
  return HLOC_OK;
}

int hloc_ws_replay(hloc_ws *ws, void *stream) {
  if (!ws) return fail(HLOC_EINVAL, "ws is NULL");
  if (!ws->exec) return fail(HLOC_ESTATE, "no batch has been captured on this workspace");
  if (ws->graph_gen != ws->db->gen)
    return fail(HLOC_ESTATE, "the database changed since the batch was captured; capture it again");
  DeviceGuard g(ws->db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipGraphLaunch(ws->exec, reinterpret_cast<hipStream_t>(stream)));
  return HLOC_OK;
}

int hloc_query_batch(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                     const int32_t *req_offsets, int32_t nreq, int32_t precision, int64_t *idx,
                     float *dist, double *xy, int32_t *tile, int32_t *flags) {
  CHK(check_query_args(db, q, nq, req_offsets, nreq, precision, idx, dist));
  CHK(check_host_offsets(req_offsets, nq, nreq, k));
  Plan p;
  CHK(make_plan(db, nq, k, n_regions, nreq, precision, &p));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  hloc_ws *ws = db->ws0;
  const bool want_agg = xy || tile || flags;
  const int64_t nqk = (int64_t)nq * k;
  CHK(ws_ensure(ws, ws->s_q, (size_t)std::max<int64_t>((int64_t)nq * db->d, 1) * sizeof(float)));
  CHK(ws_ensure(ws, ws->s_off, (size_t)(nreq + 1) * sizeof(int32_t)));
  CHK(ws_ensure(ws, ws->s_idx, (size_t)std::max<int64_t>(nqk, 1) * sizeof(int64_t)));
  CHK(ws_ensure(ws, ws->s_dist, (size_t)std::max<int64_t>(nqk, 1) * sizeof(float)));
  if (want_agg) {
    CHK(ws_ensure(ws, ws->s_xy, (size_t)std::max(nreq, 1) * 2 * sizeof(double)));
    CHK(ws_ensure(ws, ws->s_tile, (size_t)std::max(nreq, 1) * 2 * sizeof(int32_t)));
    CHK(ws_ensure(ws, ws->s_flags, (size_t)std::max(nreq, 1) * sizeof(int32_t)));
  }
  hipStream_t s = ws->stream;
  if (nq > 0)
    HIPCHK(hipMemcpyAsync(ws->s_q.p, q, (size_t)nq * db->d * sizeof(float), hipMemcpyHostToDevice, s));
  if (req_offsets)
    HIPCHK(hipMemcpyAsync(ws->s_off.p, req_offsets, (size_t)(nreq + 1) * sizeof(int32_t),
                          hipMemcpyHostToDevice, s));
  CHK(enqueue_query(ws, p, as<float>(ws->s_q), req_offsets ? as<int32_t>(ws->s_off) : nullptr,
                    nullptr, as<int64_t>(ws->s_idx), as<float>(ws->s_dist),
                    want_agg ? as<double>(ws->s_xy) : nullptr,
                    want_agg ? as<int32_t>(ws->s_tile) : nullptr,
                    want_agg ? as<int32_t>(ws->s_flags) : nullptr, s));
  if (nqk > 0) {
    HIPCHK(hipMemcpyAsync(idx, ws->s_idx.p, (size_t)nqk * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(dist, ws->s_dist.p, (size_t)nqk * sizeof(float), hipMemcpyDeviceToHost, s));
  }
  if (want_agg && nreq > 0) {
    if (xy) HIPCHK(hipMemcpyAsync(xy, ws->s_xy.p, (size_t)nreq * 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (tile) HIPCHK(hipMemcpyAsync(tile, ws->s_tile.p, (size_t)nreq * 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (flags) HIPCHK(hipMemcpyAsync(flags, ws->s_flags.p, (size_t)nreq * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return HLOC_OK;
}

int hloc_set_tiles(hloc_db *db, const hloc_tiles *tiles) {
  if (!db || !tiles) return fail(HLOC_EINVAL, "db and tiles must be non-NULL");
  const int32_t rows = tiles->rows_per_item, blocks = tiles->blocks_per_cu;
  if (rows < 16 || rows > kMaxItemRows || rows % 16 != 0)
    return fail(HLOC_EINVAL, "rows_per_item must be a multiple of 16 in 16..%d (got %d)",
                kMaxItemRows, rows);
  if (blocks < 1 || blocks > 32) return fail(HLOC_EINVAL, "blocks_per_cu must be in 1..32");
  db->tile_rows = rows;
  db->tile_blocks = blocks;
  db->chunks_fine = count_chunks(db, std::min(rows, kWideRows));
  return HLOC_OK;
}

int hloc_get_tiles(hloc_db *db, hloc_tiles *tiles) {
  if (!db || !tiles) return fail(HLOC_EINVAL, "db and tiles must be non-NULL");
  tiles->rows_per_item = db->tile_rows;
  tiles->blocks_per_cu = db->tile_blocks;
  return HLOC_OK;
}

int hloc_autotune(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                  int32_t precision, int32_t reps, hloc_tiles *best, double *best_ms) {
  if (!db || !q || !best) return fail(HLOC_EINVAL, "db, q and best must be non-NULL");
  if (nq < 1 || reps < 1) return fail(HLOC_EINVAL, "nq and reps must be >= 1");
  Plan p0;
  CHK(make_plan(db, nq, k, n_regions, nq, precision, &p0));
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  const hloc_tiles start{db->tile_rows, db->tile_blocks};
  int64_t *idx = nullptr;
  float *dist = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&](int rc) {
    if (idx) (void)hipFree(idx);
    if (dist) (void)hipFree(dist);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != HLOC_OK) (void)hloc_set_tiles(db, &start);
    return rc;
  };
  if (dev_alloc(&idx, (size_t)nq * k) || dev_alloc(&dist, (size_t)nq * k)) return cleanup(HLOC_ENOMEM);
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return cleanup(fail(HLOC_EDEVICE, "hipEventCreate failed"));
  hloc_ws *ws = db->ws0;
  const hipStream_t s = ws->stream;
  double best_t = HUGE_VAL;
  hloc_tiles bt = start;
  std::vector<float> times((size_t)reps);
  for (int32_t rows : {32, 64, 96, 128}) {
    for (int32_t blocks : {4, 8, 16}) {
      const hloc_tiles t{rows, blocks};
      int rc = hloc_set_tiles(db, &t);
      Plan p;
      if (rc == HLOC_OK) rc = make_plan(db, nq, k, n_regions, nq, precision, &p);
      // warm-up (sizes the workspace), then the timed runs
      if (rc == HLOC_OK) rc = enqueue_query(ws, p, q, nullptr, nullptr, idx, dist, nullptr, nullptr, nullptr, s);
      if (rc == HLOC_OK && hipStreamSynchronize(s) != hipSuccess) rc = fail(HLOC_EDEVICE, "warm-up failed");
      for (int32_t r = 0; rc == HLOC_OK && r < reps; ++r) {
        if (hipEventRecord(e0, s) != hipSuccess) rc = fail(HLOC_EDEVICE, "hipEventRecord failed");
        if (rc == HLOC_OK)
          rc = enqueue_query(ws, p, q, nullptr, nullptr, idx, dist, nullptr, nullptr, nullptr, s);
        if (rc == HLOC_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&times[r], e0, e1) != hipSuccess))
          rc = fail(HLOC_EDEVICE, "timing failed");
      }
      if (rc != HLOC_OK) return cleanup(rc);
      std::sort(times.begin(), times.end());
      const double med = times[times.size() / 2];
      if (med < best_t) {
        best_t = med;
        bt = t;
      }
    }
  }
  CHK(cleanup(hloc_set_tiles(db, &bt)));
  *best = bt;
  if (best_ms) *best_ms = best_t;
  return HLOC_OK;
}

int hloc_query_info(hloc_db *db, int64_t *out, int32_t n) {
  if (!db || !out || n < 0) return fail(HLOC_EINVAL, "db and out must be non-NULL, n >= 0");
  return info_of(db->ws0, out, n);
}

int hloc_ws_query_info(hloc_ws *ws, int64_t *out, int32_t n) {
  if (!ws || !out || n < 0) return fail(HLOC_EINVAL, "ws and out must be non-NULL, n >= 0");
  return info_of(ws, out, n);
}

int hloc_last_regions(hloc_db *db, int32_t *out, int32_t *nq, int32_t *n_regions_eff) {
  if (!db || !nq || !n_regions_eff) return fail(HLOC_EINVAL, "db, nq and n_regions_eff must be non-NULL");
  if (!db->has_regions) return fail(HLOC_ESTATE, "no regions");
  hloc_ws *ws = db->ws0;
  *nq = ws->last_nq;
  *n_regions_eff = ws->last_nr;
  if (!out || ws->last_nq == 0) return HLOC_OK;
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(out, ws->regions.p, (size_t)ws->last_nq * ws->last_nr * sizeof(int32_t),
                   hipMemcpyDeviceToHost));
  return HLOC_OK;
}

int hloc_profile(hloc_db *db, int32_t enable) {
  if (!db) return fail(HLOC_EINVAL, "db is NULL");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  db->ws0->prof.clear();
  db->ws0->ev_used = 0;
  db->ws0->prof_on = enable != 0;
  return HLOC_OK;
}

int hloc_profile_read(hloc_db *db, double *ms, int64_t *calls, int32_t n) {
  if (!db || !ms || !calls || n < 0) return fail(HLOC_EINVAL, "db, ms and calls must be non-NULL");
  DeviceGuard g(db->device);
  if (g.err != hipSuccess) return fail(HLOC_EDEVICE, "hipSetDevice failed");
  HIPCHK(hipDeviceSynchronize());
  hloc_ws *ws = db->ws0;
  double acc[HLOC_NUM_PHASES] = {0};
  int64_t cnt[HLOC_NUM_PHASES] = {0};
  for (const auto &r : ws->prof) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, r.a, r.b));
    acc[r.phase] += t;
    cnt[r.phase] += 1;
  }
  for (int32_t i = 0; i < std::min<int32_t>(n, HLOC_NUM_PHASES); ++i) {
    ms[i] = acc[i];
    calls[i] = cnt[i];
  }
  ws->prof.clear();
  ws->ev_used = 0;
  return HLOC_OK;
}

void hloc_free_db(hloc_db *db) {
  if (!db) return;
  {
    DeviceGuard g(db->device);
    (void)hipDeviceSynchronize();
    free_db_data(db);
  }
  delete db;
}

}  // extern "C"
