// Internal declarations shared by the hloc translation units: device buffer
// layouts, work-item format and the host-side launch wrappers of each kernel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hloc.h"

#include <algorithm>

namespace hloc {

// Event pair that times one phase of a query. While g_phase is set, every
// kernel launched through launch_kernel() is dispatched with
// hipExtLaunchKernel: the first kernel of the phase records `start` when it
// begins and each kernel records `stop` when it ends, with no extra packets
// between kernels. Set only by the query path with profiling enabled (one
// thread at a time).
struct PhaseEvents {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
  int launches = 0;
};
extern thread_local PhaseEvents *g_phase;

template <typename F, typename... Args>
inline hipError_t launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t lds, hipStream_t s,
                                Args... args) {
  if (g_phase) {
    hipEvent_t st = g_phase->launches == 0 ? g_phase->start : nullptr;
    ++g_phase->launches;
    hipExtLaunchKernelGGL(kernel, grid, block, lds, s, st, g_phase->stop, 0u, args...);
  } else {
    hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  }
  return hipGetLastError();
}

constexpr int kGroup = 16;          // frames per MFMA column block of the screen
constexpr int kLdsPerCu = 160 * 1024;  // LDS of one compute unit (gfx950)
constexpr int kItemFrames = 256;    // frames per dense work item of the wide kernels
constexpr int kListFrames = 1024;   // frames per wide list item (rows re-read once per this many)
constexpr int kWideRows = 64;       // rows per wide work item (the LDS stage of the wide kernels)
constexpr int kWideRowsRs = 128;    // rows per run of the register-row kernels (bf16, fp8)
constexpr int kWideRunsRs = 16;     // runs of kWideRowsRs rows per wide item at most
constexpr int kWideSteps = 32;      // (run, 16-frame group) steps a multi-run wide item aims at
constexpr int kMaxItemRows = 128;   // rows per narrow work item at most
constexpr int kBlock = 256;         // threads per block of most kernels
constexpr int kSelectLds = 4096;    // keys held in LDS by the select kernel
constexpr uint64_t kKeyNone = ~0ull;  // empty slot / no candidate
constexpr int kMaxSurvivors = 1024;   // want - 1 of the rerank
// Rows per block of the fine screen's output: for each frame and each 16-row
// block of its candidate rows (one MFMA tile height; a region's blocks start
// at its first row, its last block may be shorter) the fine screen writes the
// smallest screen word of the block.
constexpr int kBlockRows = 16;

inline int next_pow2_host(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// One unit of fine-screen work: rows [row_begin, row_begin + nrows) of one
// region (absolute row indices; chunk_row = offset of the chunk inside its
// region) against frames rq[q0 .. q0 + gq), gq <= kListFrames.
struct Item {
  int32_t row_begin;
  int32_t chunk_row;
  int32_t q0;
  int32_t nrows_gq;  // nrows << 16 | gq
};

// Dense or listed screen of rows against padded frames (fp32, or bf16 / fp8
// copies). Dense mode (the coarse stage) writes every screen word: frame f's
// word of row j at cand[f * cap + j]. List mode (the fine stage) writes, per
// frame, the smallest word of each 16-row block of the frame's candidate
// rows: the b-th block of a region whose blocks start at e.y in frame f's
// list goes to cand[f * cap + e.y + b].
struct ScreenArgs {
  const float *rows;      // nrows x dp, row-major
  const void *rows_lp;    // low-precision copy of rows (bf16 / fp8 screens)
  const void *q_lp;       // low-precision copy of qp
  const float *row_scale; // fp8: per-row scale
  const float *q_scale;   // fp8: per-frame scale
  const float *row_n2;    // nrows squared norms (+inf marks a row never to select)
  int32_t dp;             // padded row length (multiple of 32)
  const float *qp;        // frames x dp
  const float *qn2;       // frames squared norms
  uint32_t *cand;         // per frame: cap words (float bits of the screen distance)
  int64_t cap;            // dense: rows; list: 16-row blocks per frame at most
  int32_t rows_per_item;  // T, multiple of 16
  // dense mode: every frame against rows [0, nrows)
  int32_t dense;
  int32_t nrows;
  int32_t nq;
  // list mode
  const Item *items;
  const int32_t *n_items;
  const int2 *rq;         // (frame, offset of the region in the frame's candidate list)
  const int64_t *reg_start;
  // dense mode over a frame list (NULL: frames 0 .. nq - 1): frames
  // frame_list[0 .. *frame_count), each writing its own row of cand
  const int32_t *frame_list;
  const int32_t *frame_count;
  // register-row wide screen: 8 item counters, zero on entry, one per XCD
  // span of the items (NULL: each block takes a fixed share of its span)
  int32_t *item_ctr;
};

// Work item of the wide screens: a chunk of rows against up to kListFrames
// frames, either list item it of the narrow-then-wide order, or dense item it
// (chunk it % nchunks of all rows against frames from (it / nchunks) *
// kItemFrames).
struct WideItem {
  int row_begin, chunk_row, nrows, gq, q0, f0;
};

// Items [*lo, return value) of a wide screen launch.
__device__ __forceinline__ int wide_range(const ScreenArgs &a, int *lo) {
  if (a.dense) {
    *lo = 0;
    const int nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    return nchunks * ((a.nq + kItemFrames - 1) / kItemFrames);
  }
  *lo = a.n_items[4];
  return a.n_items[0];
}

__device__ __forceinline__ WideItem wide_item(const ScreenArgs &a, int it) {
  WideItem w;
  if (a.dense) {
    const int nchunks = (a.nrows + a.rows_per_item - 1) / a.rows_per_item;
    const int c = it % nchunks;
    w.f0 = (it / nchunks) * kItemFrames;
    w.row_begin = c * a.rows_per_item;
    w.chunk_row = w.row_begin;
    w.nrows = min(a.rows_per_item, a.nrows - w.row_begin);
    w.gq = min(kItemFrames, a.nq - w.f0);
    w.q0 = 0;
  } else {
    const Item itm = a.items[it];
    w.row_begin = itm.row_begin;
    w.chunk_row = itm.chunk_row;
    w.nrows = itm.nrows_gq >> 16;
    w.gq = itm.nrows_gq & 0xFFFF;
    w.q0 = itm.q0;
    w.f0 = 0;
  }
  return w;
}

// Frame j of a wide item (j < gq) and where its output goes: dense items,
// the word of the chunk's first row; list items, the block word of the
// chunk's first 16-row block (e is the frame's rq entry, from wide_entry).
__device__ __forceinline__ void wide_frame(const ScreenArgs &a, const WideItem &w, int j, int2 e,
                                           int *fr, int64_t *off) {
  if (a.dense) {
    *fr = w.f0 + j;
    *off = (int64_t)(*fr) * a.cap + w.chunk_row;
  } else {
    *fr = e.x;
    *off = (int64_t)e.x * a.cap + e.y + w.chunk_row / kBlockRows;
  }
}

// rq entry of frame j of a wide list item (zeros past its frames or in
// dense mode).
__device__ __forceinline__ int2 wide_entry(const ScreenArgs &a, const WideItem &w, int j) {
  return !a.dense && j < w.gq ? a.rq[w.q0 + j] : make_int2(0, 0);
}

// Per-batch counters of a workspace (cleared by the prep kernel): [0] items,
// [1] coarse fallbacks, [4] narrow items, [8] large aggregation lists, [10]
// deferred coarse frames, [16, 24) the wide screen's item counters.
constexpr int kMiscInts = 32;
constexpr int kMiscItemCtr = 16;

// Padded copy and squared norm of each frame; block 0 also clears
// zero[0 .. kMiscInts).
hipError_t launch_prep_queries(const float *q, int32_t nq, int32_t d, int32_t dp, float *qp,
                               float *qn2, int32_t *zero, hipStream_t s);
// Dense screen, or the narrow list items (every list item where no register
// kernel exists for the padded length); then the wide list items.
hipError_t launch_screen_f32(const ScreenArgs &a, int32_t grid, hipStream_t s);
// The wide kernels launch at most as many blocks as their LDS stage lets
// reside on num_cu compute units (the rest would only find no item left).
hipError_t launch_screen_wide_f32(const ScreenArgs &a, int32_t grid, int32_t num_cu, hipStream_t s);
bool f32_wide_supports(int32_t dp);  // a register wide kernel exists for this padded length
// Low-precision screens, fmt = HLOC_BF16 or HLOC_FP8.
hipError_t launch_screen_lp(int32_t fmt, const ScreenArgs &a, int32_t grid, hipStream_t s);
hipError_t launch_screen_wide_lp(int32_t fmt, const ScreenArgs &a, int32_t grid, int32_t num_cu,
                                 hipStream_t s);
bool lp_screen_supports(int32_t fmt, int32_t dp);
// The wide list items of this low-precision screen go to the register-row
// kernel: up to kWideRunsRs runs of kWideRowsRs rows each, instead of
// min(T, kWideRows) rows.
bool lp_wide_rs(int32_t fmt, int32_t dp);
// Low-precision copy of n rows (fp8: with a scale per row); maxima of the
// per-row norms of the rounding error and of the rounded row.
hipError_t launch_rows_to_lp(int32_t fmt, const float *src, int64_t n, int32_t dp, void *dst,
                             float *scale, float *max_err, float *max_norm, hipStream_t s);
// The same for the padded frames, with per-frame norms of the rounding error
// (q_err) and of the rounded frame (q_lon).
hipError_t launch_frames_to_lp(int32_t fmt, const float *qp, int32_t nq, int32_t dp, void *dst,
                               float *scale, float *q_err, float *q_lon, hipStream_t s);
// Blocks to launch for `items` work items of the screen at padded length dp.
int32_t screen_grid(int64_t items, int32_t dp, int32_t max_blocks);

// Scheduling of the fine screen.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_broadcast_ids(const int32_t *ids, int32_t nr, int32_t nq, int32_t *regions,
                                hipStream_t s);
// Work items into items[0 .. n_items[0]): narrow ones (frames of regions kept
// by at most kGroup frames) first, n_items[4] of them, then wide ones. Per
// frame f and kept-region slot j: cand_off[f][j] the first of the slot's
// 16-row blocks in the frame's block list, slot_row[f][j] the region's first
// row, slot_len[f][j] its rows; n_cand[f] the frame's block count, n_rows[f]
// its candidate rows. An rq
// entry is (frame, cand_off of the region in that frame). Narrow chunks hold
// T rows; wide chunks W rows, or with WM > 1 up to WM runs of W rows.
hipError_t launch_sched(const int32_t *regions, int32_t nq, int32_t nr, int32_t R,
                        const int64_t *reg_start, int32_t T, int32_t W, int32_t WM,
                        int32_t *rcount,
                        int32_t *rfill,
                        int32_t *vord, int32_t *rq_off, int32_t *item_off, int32_t *cand_off,
                        int32_t *slot_row, int32_t *slot_len, int32_t *n_cand, int32_t *n_rows,
                        int32_t *n_items,
                        int2 *rq, Item *items, hipStream_t s);

// Coarse screen fused with the start of the selection (coarse_gemm.hip): a
// bf16 MFMA product of frames and representatives whose epilogue keeps, per
// (frame, split of the representatives, lane group), the kCgKeep best quads
// (four consecutive representatives, ranked by their smallest screen word)
// instead of storing every word.
constexpr int kCgKeep = 6;                     // quads kept per (frame, split, lane group)
constexpr int kCgKeys = 4 * kCgKeep * 4;       // keys per (frame, split): 4 lane groups x quads x 4
struct CoarseGemmArgs {
  const void *reps;        // R x dp bf16 representatives
  const float *rep_n2;     // R squared norms (+inf: empty region)
  const void *frames;      // nq x dp bf16 frames
  const float *qn2;        // nq squared norms of the fp32 frames
  int32_t R, nq, dp;
  int32_t splits;          // representative ranges, one block column each
  int32_t reps_per_split;  // multiple of 32, splits * reps_per_split >= R
  const int32_t *rlabel;   // R region labels, or NULL (no label restriction)
  int32_t label;           // with rlabel and label_frames == 0: every frame's label
  int32_t label_frames;    // > 0: frame f's label is f / label_frames
  uint4 *slots;            // nq x splits x 4 x kCgKeep: the words of each kept quad
  uint64_t *keys;          // nq x splits x kCgKeys: (word << 32 | region), kKeyNone pads
  uint64_t *bounds;        // nq x splits x 4: per lane list, word << 32 of its last kept
                           // quad when it dropped any (every dropped region's word is at
                           // least that), else kKeyNone
};
bool coarse_gemm_supports(int32_t dp);
int32_t coarse_gemm_splits(int32_t nq, int32_t R, int32_t num_cu);
hipError_t launch_coarse_gemm(CoarseGemmArgs a, hipStream_t s);

// Per frame: the L + 1 smallest words of cand[f][0 .. n(f)) (n(f) =
// n_cand ? n_cand[f] : n_fixed; 0xFFFFFFFF entries are skipped; equal words
// ordered by position), FP64 rerank of the rows of the L smallest, top m by
// (distance, tie id), certificate against the (L + 1)-th, and the FP64
// re-score of the band of uncertain positions when it fails.
// A position is one candidate row (the coarse stage: words of
// representatives), or with `blocks` a 16-row block of the frame's candidate
// rows whose word is the smallest screen word of its rows (the fine stage):
// every row of a block is re-scored, and a block's word minus the screen's
// error bound is a lower bound of the distance of each of its rows, so the
// certificate holds per block as it does per row.
// Positions map to source rows through the frame's region slots (slot j: the
// rows from slot_row[f][j] on, at positions from slot_off[f][j] on; in block
// mode slot_len[f][j] is the slot's row count), or, with
// nslots = 0, are the rows themselves (block mode: blocks of blk_rows, every
// non-empty region in id order).
struct SelRerankArgs {
  const uint32_t *cand;
  int64_t cap;
  const int32_t *slot_off;   // nq x nslots
  const int32_t *slot_row;   // nq x nslots
  int32_t nslots;            // <= 1024
  int32_t cache;             // words kept in LDS (set by the launcher)
  const int32_t *n_cand;
  int32_t n_fixed;
  int32_t blocks;            // positions are 16-row blocks
  const int32_t *slot_len;   // block mode: nq x nslots rows of each slot's region
  const int2 *blk_rows;      // block mode, nslots = 0: (first row, rows) of each block
  int32_t L;               // positions re-scored in FP64 (rows: <= kMaxSurvivors)
  int32_t m;               // results per frame (<= 256, <= L)
  const float *src32;      // fp32 source rows (fine stage) or NULL
  const double *src64;     // fp64 source rows (coarse stage) or NULL
  int32_t dp;
  const int32_t *tie_of;   // source row -> original index; NULL: the row id itself
  const float *qp;         // frames x dp padded fp32
  const float *qn2;
  double err_coef;         // screen error bound: err_coef * (|q| + max_norm)^2
  double max_norm;
  // low-precision screen: + lo_coef * (|q~| lo_dmax + |q~ - q| lo_nmax + |q~ - q| lo_dmax)
  const float *q_err;      // per frame |q~ - q| (NULL: fp32 screen)
  const float *q_lon;      // per frame |q~|
  double lo_dmax;          // largest |d~ - d| over the rows
  double lo_nmax;          // largest |d~|
  double lo_coef;
  int32_t nq;
  int64_t *idx_out;        // fine: nq x m original indices
  float *dist_out;         // fine: nq x m
  int32_t *reg_out;        // coarse: nq x m region ids
  int32_t *stat_fallback;  // count of frames whose certificate failed (or NULL)
  // per frame, written once by the frame's block or wave (or NULL): candidate
  // count, rows re-scored in FP64 (survivors and band), band rows, flags (1:
  // the certificate failed and the band was re-scored, 2: in several chunks).
  // Plain stores: one counter shared by every frame would serialise at L2.
  int4 *frame_stat;
  // key mode (the coarse stage after the fused coarse product): the frame's
  // n_fixed candidates are keys (word << 32 | source row, any order), and
  // n_bounds bounds per frame: every source row missing from the keys has a
  // key of at least their minimum. A frame whose keys cannot decide the
  // selection writes nothing: it is appended to defer_list (count in
  // *defer_count, zero on entry) for the dense screen and words mode.
  const uint64_t *keys;    // nq x n_fixed, or NULL (words mode)
  const uint64_t *bounds;  // nq x n_bounds
  int32_t n_bounds;
  int32_t *defer_list;     // nq entries
  int32_t *defer_count;
  // words mode over a frame list (NULL: block b takes frame b in XCD-major
  // order): block b < *frame_count takes frame frame_list[b]
  const int32_t *frame_list;
  const int32_t *frame_count;
};
hipError_t launch_select_rerank(SelRerankArgs a, hipStream_t s);

// Aggregation (Algorithm 2) per request.
struct AggArgs {
  const int64_t *idx;        // nq x k
  int32_t k;
  int32_t nq;
  const int32_t *req_offsets;  // nreq + 1 or NULL (one frame per request)
  const int32_t *req_k;      // per request: candidates per frame pooled (<= k), or NULL (k)
  int32_t nreq;
  const int2 *tile_of;       // original index -> (ix, iy)
  double cell;
  int32_t top_c;
  int32_t rho;
  int32_t toler_pct;
  double *xy;
  int32_t *tile;
  int32_t *flags;
  int32_t *big_list;   // nreq: requests pooling more than 512 candidates
  int32_t *big_count;  // zero on entry
  int32_t num_cu;
};
hipError_t launch_aggregate(const AggArgs &a, hipStream_t s);

// Kernel attributes (LDS limits) for the current device; called once when a
// database is built so that no attribute is set while a graph is captured.
hipError_t prepare_screen_kernels();  // also the low-precision screens
hipError_t prepare_screen_lp_kernels();
hipError_t prepare_select_kernels();
hipError_t prepare_aggregate_kernels();
hipError_t prepare_sched_kernels();
hipError_t prepare_coarse_gemm_kernels();
inline hipError_t prepare_kernels() {
  hipError_t e = prepare_screen_kernels();
  if (e == hipSuccess) e = prepare_coarse_gemm_kernels();
  if (e == hipSuccess) e = prepare_select_kernels();
  if (e == hipSuccess) e = prepare_sched_kernels();
  if (e == hipSuccess) e = prepare_aggregate_kernels();
  return e;
}

// Database set-up.
hipError_t launch_gather_rows(const float *src, const int32_t *src_row, int64_t n, int32_t d,
                              int32_t src_stride, float *dst, int32_t dp, hipStream_t s);
hipError_t launch_row_norms(const float *rows, int64_t n, int32_t dp, float *n2,
                            float *max_norm, hipStream_t s);
hipError_t launch_region_means(const float *rows, const int64_t *reg_start, int32_t R,
                               int32_t dp, double *mean64, hipStream_t s);
hipError_t launch_rep_finish(const double *rep64, const int64_t *reg_start, int32_t R,
                             int32_t dp, float *rep32, float *rep_n2, float *max_norm,
                             hipStream_t s);
hipError_t launch_tiles(const double *xy, int64_t n, double cell, int2 *tile, hipStream_t s);

}  // namespace hloc
