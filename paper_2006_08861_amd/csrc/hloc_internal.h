// Internal declarations shared by the hloc translation units: device buffer
// layouts, work-item format and the host-side launch wrappers of each kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hloc {

constexpr int kGroup = 16;          // frames per MFMA column block of the screen
constexpr int kBlock = 256;         // threads per block of most kernels
constexpr int kSelectLds = 4096;    // keys held in LDS by the select kernel
constexpr uint64_t kKeyNone = ~0ull;  // empty slot / no candidate
constexpr int kMaxSurvivors = 1024;   // want - 1 of the rerank

inline int next_pow2_host(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// One unit of fine-screen work: rows [chunk_row, chunk_row + T) of `region`
// (clipped to the region) against frames rq[q0 .. q0 + gq).
struct Item {
  int32_t region;
  int32_t chunk_row;  // first row of the chunk, relative to the region start
  int32_t q0;
  int32_t gq;
};

// Dense or listed screen of fp32 rows against padded fp32 frames.
struct ScreenF32Args {
  const float *rows;      // nrows x dp, row-major
  const float *row_n2;    // nrows squared norms (+inf marks a row never to select)
  int32_t dp;             // padded row length (multiple of 32)
  const float *qp;        // frames x dp
  const float *qn2;       // frames squared norms
  uint64_t *cand;         // per frame: cap keys (dist bits << 32 | row)
  int64_t cap;
  int32_t rows_per_item;  // T, multiple of 64
  // dense mode: every frame against rows [0, nrows)
  int32_t dense;
  int32_t nrows;
  int32_t nq;
  // list mode
  const Item *items;
  const int32_t *n_items;
  const int2 *rq;         // (frame, offset of the region in the frame's candidate list)
  const int64_t *reg_start;
};

hipError_t launch_prep_queries(const float *q, int32_t nq, int32_t d, int32_t dp, float *qp,
                               float *qn2, hipStream_t s);
hipError_t launch_screen_f32(const ScreenF32Args &a, int32_t grid, hipStream_t s);

// Scheduling of the fine screen.
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_broadcast_ids(const int32_t *ids, int32_t nr, int32_t nq, int32_t *regions,
                                hipStream_t s);
hipError_t launch_sched(const int32_t *regions, int32_t nq, int32_t nr, int32_t R,
                        const int64_t *reg_start, int32_t T, int32_t *rcount, int32_t *rfill,
                        int32_t *rq_off, int32_t *item_off, int32_t *cand_off, int32_t *n_cand,
                        int32_t *n_items, int2 *rq, Item *items, hipStream_t s);

// Per-frame selection of the `want` smallest keys of cand[q][0 .. n(q)).
// n(q) = n_cand ? n_cand[q] : n_fixed. Output sel[q][want], ascending,
// kKeyNone-padded.
hipError_t launch_select(const uint64_t *cand, int64_t cap, const int32_t *n_cand,
                         int32_t n_fixed, int32_t nq, int32_t want, uint64_t *sel,
                         int32_t *stat_max_cand, hipStream_t s);

// FP64 rerank of the survivors and certificate against the best rejected
// screen distance.
struct RerankArgs {
  const uint64_t *sel;     // nq x want sorted keys; key low word = source row
  int32_t want;            // survivors + 1
  int32_t m;               // results per frame
  const int32_t *n_cand;   // per-frame candidate count (NULL: n_fixed)
  int32_t n_fixed;
  const float *src32;      // fp32 source rows (stage 2) or NULL
  const double *src64;     // fp64 source rows (stage 1) or NULL
  int32_t dp;
  const int32_t *tie_of;   // source row -> tie id (original index); NULL: the row itself
  const float *qp;         // frames x dp padded fp32
  const float *qn2;
  double err_coef;         // screen error bound: err_coef * (|q| + max_norm)^2
  double max_norm;
  int32_t nq;
  int64_t *idx_out;        // stage 2: nq x m original indices
  float *dist_out;         // stage 2: nq x m
  int32_t *reg_out;        // stage 1: nq x m ids
  int32_t *flag;           // per frame: 1 = not certified
  int32_t *stat_fallback;  // counter of uncertified frames
};
hipError_t launch_rerank(const RerankArgs &a, hipStream_t s);

// Exact FP64 recomputation over a frame's whole candidate set, for frames
// whose rerank was not certified.
struct ExactArgs {
  const int32_t *flag;
  int32_t nq;
  int32_t m;
  int32_t dp;
  const float *qp;
  // stage 2: candidate rows are the frame's regions, in list order
  const float *src32;
  const int32_t *regions;  // nq x nr
  int32_t nr;
  const int32_t *cand_off; // nq x nr: first candidate position of each kept region
  const int32_t *n_cand;   // nq
  const int64_t *reg_start;
  const int32_t *tie_of;   // row -> original index
  int64_t *idx_out;
  float *dist_out;
  // stage 1: candidate rows are all regions 0..R-1 of src64 (empty skipped)
  const double *src64;
  int32_t R;
  int32_t *reg_out;
};
hipError_t launch_exact(const ExactArgs &a, hipStream_t s);

// Aggregation (Algorithm 2) per request.
struct AggArgs {
  const int64_t *idx;        // nq x k
  int32_t k;
  int32_t nq;
  const int32_t *req_offsets;  // nreq + 1 or NULL (one frame per request)
  int32_t nreq;
  const int2 *tile_of;       // original index -> (ix, iy)
  double cell;
  int32_t top_c;
  int32_t rho;
  int32_t toler_pct;
  double *xy;
  int32_t *tile;
  int32_t *flags;
};
hipError_t launch_aggregate(const AggArgs &a, hipStream_t s);

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
