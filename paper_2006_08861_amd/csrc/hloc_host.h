// Host-side internals shared by the C ABI (hloc_api.hip) and the request
// server (server.hip): the database and workspace structures, the plan of a
// batch and the sequence of kernels that localizes it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "hloc.h"
#include "hloc_internal.h"

namespace hloc {

// Sets the calling thread's hloc_last_error message; returns code.
int fail(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess) return fail(HLOC_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)                   \
  do {                              \
    int rc_ = (expr);               \
    if (rc_ != HLOC_OK) return rc_; \
  } while (0)

struct DeviceGuard {
  int old = -1;
  hipError_t err;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

struct WsBuf {
  void *p = nullptr;
  size_t cap = 0;
};

constexpr int kRegionMargin = 4;    // extra regions re-scored in FP64 by the coarse stage
constexpr int kOversample = 16;     // extra rows re-scored in FP64 by the fine stage
constexpr int kRowsCoarse = 64;     // rows (representatives) per coarse work item
constexpr int kRowsFine = 64;       // rows per fine work item
constexpr int kWideDenseFrames = 512;  // batches from which the coarse screen uses the wide kernels
constexpr double kUnit32 = 5.9604644775390625e-08;  // 2^-24

template <class T>
T *as(WsBuf &b) {
  return reinterpret_cast<T *>(b.p);
}

struct ProfRec {
  int phase;
  hipEvent_t a, b;
};

// A low-precision copy of the rows and the representatives (bf16, or fp8 with
// a scale per vector) and the largest norms of its rounding errors and of the
// rounded vectors.
struct LpMirror {
  void *rows = nullptr;
  float *scale = nullptr;
  void *reps = nullptr;
  float *rep_scale = nullptr;
  float err = 0.f, norm = 0.f, rep_err = 0.f, rep_norm = 0.f;
};

// Bytes per value of a low-precision format (HLOC_BF16 / HLOC_FP8).
inline int lp_bytes(int fmt) { return fmt == HLOC_BF16 ? 2 : 1; }

constexpr int kNormSlots = 10;  // largest-norm slots of a database (see hloc_db)

}  // namespace hloc

// Scratch memory, counters, profile record and captured graph of one batch in
// flight. Batches on distinct workspaces may overlap on the device.
struct hloc_ws {
  hloc_db *db = nullptr;
  hipStream_t stream = nullptr;  // own stream (graph capture, host-pointer calls)
  hloc::WsBuf qp, qn2, cand1, regions, rcount, rfill, vord, rq_off, item_off, cand_off, n_cand, misc, rq,
      items, cand2, agg_xy, agg_tile, agg_flags, q_lp, q_scale, q_err, q_lon, slot_row, slot_len, n_rows,
      fstat,                        // fine select's per-frame statistics
      c_lp, c_scale, c_err, c_lon,  // bf16 frame copy for the coarse screen of fp8 queries
      agg_big,                      // requests for the large-list aggregation kernel
      lab_off, lab_list,            // frame lists of a query over subspace labels
      lab_q,                        // its frames once per label
      ckeys, cslots, cbounds,       // key lists of the fused coarse product
      cdefer;                       // frames its keys could not decide
  hloc::WsBuf s_q, s_off, s_idx, s_dist, s_xy, s_tile, s_flags;  // staging of host-pointer calls
  int32_t last_nq = 0, last_nr = 0, last_kp = 0;
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<hloc::ProfRec> prof;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t graph_gen = 0;  // hloc_db::gen when the graph was captured
};

struct hloc_db {
  int device = 0;
  int num_cu = 256;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int32_t d = 0, dp = 0;
  float *rows = nullptr;      // n x dp fp32, region-contiguous once regions are set
  float *row_n2 = nullptr;    // n squared norms
  int32_t *perm = nullptr;    // device row -> original index
  double *xy = nullptr;       // n x 2 by original index
  int2 *tiles = nullptr;      // n by original index
  // largest norms: [0] rows, [1] representatives, then for format f (1 bf16,
  // 2 fp8) at 4 f - 2: rounding error of the rows, rounded rows, rounding
  // error of the representatives, rounded representatives
  float *norm_max = nullptr;
  float h_row_max = 0.f, h_rep_max = 0.f;
  uint32_t mirrors = 0;        // HLOC_MIRROR_* copies kept beside the fp32 rows
  hloc::LpMirror lp[3];        // [HLOC_BF16], [HLOC_FP8]
  std::vector<int32_t> h_perm;
  double max_abs_coord = 0.0;
  bool has_regions = false;
  int32_t R = 0, R_nonempty = 0;
  int64_t max_region = 0;
  int64_t *reg_start = nullptr;
  std::vector<int64_t> h_reg_start;
  std::vector<int64_t> h_desc_prefix;  // sum of the j largest region sizes, j = 0..R
  std::vector<int64_t> h_desc_blocks;  // sum of the j largest regions' 16-row block counts
  int64_t n_blocks = 0;                // 16-row blocks over all regions
  int2 *blk_rows = nullptr;            // per block, regions in id order: (first row, rows)
  int64_t chunks_fine = 0;             // sum over regions of ceil(size / min(tile_rows, 64))
  int32_t tile_rows = hloc::kRowsFine; // rows per narrow fine work item (multiple of 16, <= 128)
  int32_t tile_blocks = 8;             // blocks per compute unit of the screen launches
  int32_t *nonempty_ids = nullptr;
  double *rep64 = nullptr;
  float *rep32 = nullptr;
  float *rep_n2 = nullptr;
  double cell = 0.5, radius = 0.0;
  int32_t top_c = 1, rho = 0, pct = 0;
  int32_t *rlabel = nullptr;             // subspace label of each region (R), or NULL
  int32_t n_labels = 0;
  std::vector<int32_t> h_label_nonempty;  // non-empty regions per label
  hloc_ws *ws0 = nullptr;  // workspace of the calls that take no workspace
  int32_t user_ws = 0;     // workspaces created by the caller and not yet freed
  int32_t servers = 0;     // request servers over this database not yet freed
  uint64_t gen = 1;        // bumped whenever arrays or constants a captured graph uses change
};

namespace hloc {

struct Plan {
  int32_t nq, k, nr, L1, kp, nreq, precision;
  bool exhaustive;
  // the coarse stage as the fused bf16 product (short key lists per frame)
  // instead of the dense screen's frame x region words
  bool coarse_keys;
  int32_t csplits, creps;  // representative ranges and their length
  int64_t cap2;  // 16-row blocks of a frame's candidate rows at most
  int64_t items_bound;
  int32_t grid1, grid2;
};

void free_buf(WsBuf &b);
// Grows b to at least bytes (waits for the device first: the old buffer may
// be in use).
int ensure(WsBuf &b, size_t bytes);
// ensure() for a buffer of ws: a reallocation drops the graph captured on ws
// (it holds the old address).
int ws_ensure(hloc_ws *ws, WsBuf &b, size_t bytes);
void drop_graph(hloc_ws *ws);
int make_plan(const hloc_db *db, int32_t nq, int32_t k, int32_t n_regions, int32_t nreq,
              int32_t precision, Plan *pl);
// Bytes ensure() allocates for a request of `bytes`.
size_t alloc_size(size_t bytes);
// Memory the workspace buffers are carved from instead of allocated.
struct Carve {
  void *base;
};
// Sizes every buffer of ws for plan p (agg_internal: the aggregation outputs
// live in the workspace). With `bytes` set, allocates nothing and adds to
// *bytes what sizing an empty workspace would allocate; with `carve` too,
// points every buffer into carve->base from offset *bytes on (each exactly
// its size, 256-byte aligned) and advances *bytes past them.
int ensure_workspace(hloc_ws *ws, const Plan &p, bool agg_internal, size_t *bytes = nullptr,
                     const Carve *carve = nullptr);
// Enqueues one batch on stream s. req_k (device, nreq entries, or NULL) gives
// each request's candidates per frame for the aggregation (<= p.k).
// req_frames (device, n_frames entries, or NULL): request r pools the batch
// frames req_frames[req_offsets[r] .. req_offsets[r+1]-1] instead of the
// frames req_offsets[r] .. req_offsets[r+1]-1.
// label >= 0: the coarse selection keeps only regions with that label;
// label_frames > 0: frame f keeps only regions labelled f / label_frames.
int enqueue_query(hloc_ws *ws, const Plan &p, const float *q, const int32_t *req_offsets,
                  const int32_t *req_k, int64_t *idx, float *dist, double *xy, int32_t *tile,
                  int32_t *flags, hipStream_t s, const int32_t *req_frames = nullptr,
                  int32_t n_frames = 0, int32_t label = -1, int32_t label_frames = 0);
hipError_t launch_mask_label(uint32_t *words, int32_t nq, int32_t R, const int32_t *rlabel,
                             int32_t p, int32_t per, hipStream_t s);
hipError_t launch_label_lists(const int32_t *req_offsets, int32_t nreq, int32_t nq, int32_t P,
                              int32_t *list_off, int32_t *list, hipStream_t s);
// The aggregation of aggregate.hip over a frame list (NULL: contiguous frames).
hipError_t launch_aggregate_frames(const AggArgs &a, const int32_t *frames, int32_t n_frames,
                                   hipStream_t s);
int check_query_args(const hloc_db *db, const float *q, int32_t nq, const int32_t *req_offsets,
                     int32_t nreq, int32_t precision, const int64_t *idx, const float *dist);
int new_ws(hloc_db *db, hloc_ws **out);
void free_ws(hloc_ws *ws);

}  // namespace hloc
