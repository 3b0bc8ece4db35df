/*
 * hloc — hierarchical L2 retrieval and 2-D candidate aggregation for indoor
 * localization, on AMD Instinct MI355X (gfx950).
 *
 * Method: Hu, Zhu, Zhang, "GPU-accelerated Hierarchical Panoramic Image Feature
 * Retrieval for Indoor Localization", ICMR 2016.
 *   - Database of feature vectors with a geo-referenced (x, y) per entry:
 *     Section 3 (environment modeling) and Section 3.2 (mapping table).
 *   - Subspaces searched in parallel, each frame compared with every database
 *     frame by Euclidean distance, top-N candidates per frame: Section 3.1,
 *     Algorithm 1, Section 4. Here the database is split into regions with a
 *     coarse representative each; a frame searches every row of its best
 *     `n_regions` regions (all regions = the paper's exhaustive search).
 *   - Multi-frame requests and 2-D density aggregation: Section 3.1 and
 *     Section 3.2, Algorithm 2.
 *   - The feature itself, the Fourier magnitude of a 1-D panoramic signal:
 *     Section 3 (hloc_fft_features_async).
 *
 * Conventions for every call:
 *   - Return value: HLOC_OK (0) or a negative hloc_status. On error the
 *     outputs are unspecified and hloc_last_error() describes the failure.
 *   - Ownership: the caller owns every buffer it passes. The library copies
 *     database inputs during the call and keeps no caller pointer afterwards.
 *   - Threads: calls on one hloc_db must not overlap (the database owns one
 *     default workspace). Batches on distinct workspaces (hloc_ws) of one
 *     database may be in flight at the same time on different streams.
 *     Distinct databases are independent.
 *   - Devices: a database lives on the HIP device that was current when it
 *     was built; later calls make that device current.
 */
#ifndef HLOC_H
#define HLOC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hloc_db hloc_db; /* opaque; owns all of its device memory */
typedef struct hloc_ws hloc_ws; /* opaque; scratch memory of one batch in flight */
typedef struct hloc_server hloc_server; /* opaque; request loop over one database */

typedef enum {
  HLOC_OK = 0,
  HLOC_EINVAL = -1,      /* an argument is out of range or malformed */
  HLOC_ENOMEM = -2,      /* device or host allocation failed */
  HLOC_ESTATE = -3,      /* call order violated (e.g. query before set_regions) */
  HLOC_EDEVICE = -4,     /* a HIP call failed; the message names it */
  HLOC_EUNSUPPORTED = -5, /* the requested screen precision is not available */
  HLOC_EBUSY = -6,       /* the request server's queue is full; submit again later */
  HLOC_ETIMEDOUT = -7    /* the wait ended before the request completed */
} hloc_status;

/* Precision of the screens. HLOC_BF16 screens rows and region
 * representatives from bf16 copies (database built with HLOC_MIRROR_BF16),
 * HLOC_FP8 from OCP e4m3 copies with one fp32 scale per vector (max |v| / 448;
 * database built with HLOC_MIRROR_FP8; padded length a multiple of 64).
 * Whatever the screen, the returned top-k is decided by an FP64 rerank of the
 * survivors (k + 16 of them behind fp32, 3k behind bf16 and fp8) and the
 * regions by an FP64 re-score of the best n_regions + 4, each with a
 * certificate: candidates the screen's error bound cannot exclude are
 * re-scored too, so the result is the same for every precision (a looser
 * bound only costs more re-scoring). */
typedef enum { HLOC_FP32 = 0, HLOC_BF16 = 1, HLOC_FP8 = 2 } hloc_precision;

/* Per-request flags written by the aggregation (bit set). */
enum {
  HLOC_FLAG_LOW_CONFIDENCE = 1, /* no TopC tile passed the threshold; rank-1 tile returned */
  HLOC_FLAG_EMPTY = 2,          /* request had no candidate; position is NaN */
  HLOC_FLAG_BAD_REQUEST = 4     /* offsets not monotone / out of range, or too many candidates */
};

/* Low-precision copies of the rows kept beside the fp32 rows (build flags). */
enum { HLOC_MIRROR_BF16 = 1, HLOC_MIRROR_FP8 = 2 };

/* Limits. */
#define HLOC_MAX_DIM 1024            /* d */
#define HLOC_MAX_K 256               /* k */
#define HLOC_MAX_REQUEST_CANDIDATES 4096 /* frames of one request x k */
#define HLOC_MAX_TOP_C 64
#define HLOC_MAX_LABELS 64           /* subspace labels */
#define HLOC_STATIC_SCRATCH_BYTES 67108864 /* scratch of hloc_query_batch_static_async (64 MiB) */

/*
 * Build a database from n feature vectors (Section 3: one omnidirectional
 * feature per modeled frame) and their floor-plan positions (Section 3.2: the
 * geo-referenced mapping table).
 *   feats : host, n x d float32, row-major, every value finite.
 *   xy    : host, n x 2 float64 metres (x west->east, y south->north), finite.
 *   n     : 1 .. 2^31-1 rows;  d : 1 .. HLOC_MAX_DIM.
 *   mirrors: HLOC_MIRROR_* bits: HLOC_MIRROR_BF16 keeps a bf16 copy of the rows
 *            (half the bytes) for the HLOC_BF16 screen, HLOC_MIRROR_FP8 an
 *            e4m3 copy with a scale per row (a quarter) for HLOC_FP8; 0 for
 *            fp32 only.
 *   out   : receives the new handle (set to NULL on error).
 * Errors: EINVAL (sizes, NULL pointers, non-finite values), EUNSUPPORTED
 * (unknown mirror flag), ENOMEM, EDEVICE.
 * The database is not queryable until hloc_set_regions() succeeds.
 */
int hloc_build_db(const float *feats, int64_t n, int32_t d, const double *xy, uint32_t mirrors,
                  hloc_db **out);

/*
 * Partition the rows into regions (the subspaces of Section 3.1) and compute
 * each region's representative.
 *   region_of : host, n int32 in [0, n_regions_total).
 *   reps      : host, n_regions_total x d float32 representatives, or NULL to
 *               use each region's mean row (computed in FP64 on the device).
 * Regions with no row are never selected. Rows are re-laid out
 * region-contiguously on the device. Errors: EINVAL, ENOMEM, EDEVICE.
 */
int hloc_set_regions(hloc_db *db, const int32_t *region_of, int32_t n_regions_total,
                     const float *reps);

/*
 * Aggregation constants of Algorithm 2 (Section 3.2): tile edge cell_m > 0,
 * top_c in 1 .. HLOC_MAX_TOP_C, tolerance-circle radius radius_m >= 0 (in
 * whole tiles: rho = round(radius_m / cell_m)), threshold toler_pct in
 * 0 .. 100. The paper uses 0.30 m, 10, 3 m, 20 %. Default until called:
 * argmax of a 0.5 m grid (0.5, 1, 0, 0). Errors: EINVAL (also when a
 * position is beyond 2^30 tiles from the origin), EDEVICE.
 */
int hloc_set_aggregation(hloc_db *db, double cell_m, int32_t top_c, double radius_m,
                         int32_t toler_pct);

/*
 * Localize a batch (host pointers; blocks until done).
 *   q           : nq x d float32 query frames, row-major (nq >= 0).
 *   k           : 1 .. HLOC_MAX_K candidates per frame.
 *   n_regions   : >= 1 regions searched per frame; clamped to the number of
 *                 non-empty regions.
 *   req_offsets : nreq + 1 int32, non-decreasing, from 0 to nq: request i owns
 *                 frames [req_offsets[i], req_offsets[i+1]). NULL means one
 *                 frame per request (nreq must equal nq).
 *   precision   : hloc_precision of the screen.
 * Outputs (row-major):
 *   idx   : nq x k int64 original row indices by (squared distance, index)
 *           ascending; -1 where fewer than k candidates exist.
 *   dist  : nq x k float32 squared L2 distances (FP64 rounded), +inf padding.
 *   xy    : nreq x 2 float64 estimate (tile centre), or NULL.
 *   tile  : nreq x 2 int32 (ix, iy) of the estimate, or NULL.
 *   flags : nreq int32 HLOC_FLAG_* bits, or NULL.
 * If xy, tile and flags are all NULL the aggregation is skipped.
 * Errors: EINVAL, ESTATE (no regions yet), EUNSUPPORTED, ENOMEM, EDEVICE.
 */
int hloc_query_batch(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                     const int32_t *req_offsets, int32_t nreq, int32_t precision, int64_t *idx,
                     float *dist, double *xy, int32_t *tile, int32_t *flags);

/*
 * Same as hloc_query_batch, but every pointer is device memory on the
 * database's device and the work is enqueued on `stream` (a hipStream_t; NULL
 * is the null stream); the call returns without waiting. Pointers must stay
 * valid until the stream passes the call. Malformed req_offsets are not
 * detected on the host: the affected requests get HLOC_FLAG_BAD_REQUEST.
 * The call may allocate (grow the workspace) unless hloc_reserve() sized it
 * beforehand.
 */
int hloc_query_batch_async(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                           const int32_t *req_offsets, int32_t nreq, int32_t precision,
                           int64_t *idx, float *dist, double *xy, int32_t *tile, int32_t *flags,
                           void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as hloc_query_batch_async, same arguments, outputs and errors, with
 * bitwise the same results, but it allocates nothing. The batch's scratch
 * memory (frame copies, screen words, schedule, counters) is carved from a
 * static device array of HLOC_STATIC_SCRATCH_BYTES that every device the
 * library runs on holds from the first call on that device until the process
 * ends; only the caller's inputs and outputs are passed in.
 * Errors as hloc_query_batch_async, plus EINVAL when the batch's scratch
 * memory would exceed HLOC_STATIC_SCRATCH_BYTES (the message gives the size
 * needed; e.g. 256 frames against 1,024 regions need about 2 MB) and EDEVICE
 * when the array's device address cannot be looked up.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (the kernels clear what must start at zero): calls on one
 * device whose work overlaps on the GPU race, so enqueue them on one stream
 * or wait for the previous one first. hloc_query_info does not report on
 * these calls.
 */
int hloc_query_batch_static_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                                  int32_t n_regions, const int32_t *req_offsets, int32_t nreq,
                                  int32_t precision, int64_t *idx, float *dist, double *xy,
                                  int32_t *tile, int32_t *flags, void *stream);

/*
 * Sliding-window requests (Section 3.1: a request carries a frame and its
 * neighbours, so consecutive requests of a video share all but one frame).
 * Every frame of the batch is retrieved once; request i pools the results of
 * the batch frames req_frames[req_offsets[i] .. req_offsets[i+1]-1] (indices
 * into q, any order, repeats pooled again) and is aggregated as in
 * hloc_query_batch. Device pointers, enqueued on `stream` like
 * hloc_query_batch_async.
 *   req_offsets : nreq + 1 int32 (device), non-decreasing from 0 to n_list.
 *   req_frames  : n_list int32 (device), each in [0, nq).
 * Outputs as hloc_query_batch (idx / dist per frame, xy / tile / flags per
 * request). Malformed offsets or an index outside [0, nq) are detected on the
 * device: that request gets HLOC_FLAG_BAD_REQUEST.
 * Errors: EINVAL (NULL lists with nreq > 0, n_list < 0, as hloc_query_batch),
 * ESTATE, EUNSUPPORTED, ENOMEM, EDEVICE.
 */
int hloc_query_windows_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                             int32_t n_regions, const int32_t *req_offsets,
                             const int32_t *req_frames, int32_t n_list, int32_t nreq,
                             int32_t precision, int64_t *idx, float *dist, double *xy,
                             int32_t *tile, int32_t *flags, void *stream);

/*
 * Sliding windows across calls (Section 3.1: the request for frame q_m
 * carries the frames before it; M = 11 in Section 4). A video stream sends
 * each frame once: the library keeps, per stream, the top-k lists of its
 * last window - 1 frames on the device, and the estimate of a new frame
 * pools its own list with those (its window), so every frame is retrieved
 * once however many windows it belongs to.
 *
 * hloc_streams_create: state for n_streams streams (ids 0 .. n_streams - 1),
 * windows of `window` frames (window x k <= HLOC_MAX_REQUEST_CANDIDATES), k
 * candidates per frame and at most max_frames new frames per call; device
 * memory about (n_streams (window - 1) + max_frames) k 8 bytes. Every stream
 * starts empty. The state holds a workspace of db until hloc_streams_free.
 * hloc_streams_reset forgets every stream's frames (waits for the device).
 *
 * hloc_query_streams_async: new frames q (nq x d, device) in nseg segments:
 * segment g is frames seg_offsets[g] .. seg_offsets[g+1]-1 of stream
 * seg_stream[g], in capture order (device arrays of nseg + 1 and nseg
 * int32; a stream in at most one segment per call). Per new frame: its top-k
 * (idx / dist, nq x k, or both NULL) and the estimate of its window (xy,
 * tile, flags, nq entries): the frame and the frames before it in its stream,
 * from this call and earlier calls, at most `window` of them, aggregated as
 * in hloc_query_batch. Afterwards each stream in the call keeps its last
 * window - 1 frames. A segment whose stream is out of range, repeated in the
 * call, or whose offsets are malformed is ignored (its frames get
 * HLOC_FLAG_BAD_REQUEST and its stream is left as it was), as are frames
 * outside every segment. Enqueued on `stream`; calls on one state must be
 * ordered (one stream, or waited for). Every frame of the batch is retrieved
 * with n_regions and precision as in hloc_query_batch.
 * Errors: EINVAL (sizes, NULL pointers, nq > max_frames, window x k too
 * large), ENOMEM, ESTATE, EUNSUPPORTED, EDEVICE.
 */
typedef struct hloc_streams hloc_streams;
int hloc_streams_create(hloc_db *db, int32_t n_streams, int32_t window, int32_t k,
                        int32_t max_frames, hloc_streams **out);
int hloc_streams_reset(hloc_streams *st);
void hloc_streams_free(hloc_streams *st);
int hloc_query_streams_async(hloc_streams *st, const float *q, int32_t nq, int32_t n_regions,
                             int32_t precision, const int32_t *seg_offsets,
                             const int32_t *seg_stream, int32_t nseg, int64_t *idx, float *dist,
                             double *xy, int32_t *tile, int32_t *flags, void *stream);

/*
 * Subspace labels (Section 3.1: the database is split into subspaces, such as
 * the walked paths of Section 4, where the top N candidates of every path are
 * kept: N x M x P for a request of M frames over P paths). labels: host, one
 * int32 per region (R of hloc_set_regions), each in [0, n_labels); every
 * label needs a non-empty region. Copied; hloc_set_regions drops them.
 * Errors: EINVAL, ESTATE (no regions yet, or a server uses the database),
 * ENOMEM, EDEVICE.
 */
int hloc_set_region_labels(hloc_db *db, const int32_t *labels, int32_t n_labels);

/*
 * Top k per (frame, label) and the aggregation over all of them: for every
 * label p, each frame runs the search of hloc_query_batch restricted to the
 * regions labelled p (the best min(n_regions, regions of p) of them, then their
 * rows); request i pools, for each of its frames and each label, the k
 * results (frames x labels x k candidates, at most
 * HLOC_MAX_REQUEST_CANDIDATES). Device pointers, enqueued on `stream`.
 *   n_labels    : the label count given to hloc_set_region_labels (the
 *                 caller's outputs are sized by it; a different value is
 *                 EINVAL, so the kernels never write past them).
 *   req_offsets : nreq + 1 int32 (device) as hloc_query_batch, or NULL.
 *   idx, dist   : n_labels x nq x k (label-major), as hloc_query_batch.
 *   xy, tile, flags : per request, required when nreq > 0.
 * Errors: EINVAL, ESTATE (no labels), EUNSUPPORTED, ENOMEM, EDEVICE.
 */
int hloc_query_labels_async(hloc_db *db, const float *q, int32_t nq, int32_t k,
                            int32_t n_regions, int32_t n_labels, const int32_t *req_offsets,
                            int32_t nreq,
                            int32_t precision, int64_t *idx, float *dist, double *xy,
                            int32_t *tile, int32_t *flags, void *stream);

/*
 * Pre-size the workspace for batches up to nq_max frames, nreq_max requests,
 * k_max and n_regions_max, so that later query calls within these limits
 * allocate nothing. Errors: EINVAL, ESTATE, ENOMEM, EDEVICE.
 */
int hloc_reserve(hloc_db *db, int32_t nq_max, int32_t nreq_max, int32_t k_max,
                 int32_t n_regions_max);

/*
 * Per-database counters of the last query call (waits for it): out[0] work
 * items of the fine screen, out[1] frames whose coarse selection failed its
 * certificate (so the band of uncertain regions was re-scored in FP64),
 * out[2] frames whose top-k did (the band of uncertain rows), out[3] largest
 * count of 16-row candidate blocks of a frame, out[4] survivor rows per
 * frame (k'), out[5] total candidate rows screened, out[6] narrow work items
 * (regions kept by at most 16 frames; out[0] - out[6] are wide items),
 * out[7] frames whose band was too large for one pass and was re-scored in
 * chunks, out[8] row slots re-scored in bands over all frames (16 per
 * block), out[9] row slots re-scored in FP64 by the fine stage over all
 * frames (survivor blocks and bands), out[10] frames whose coarse
 * selection the fused coarse product's kept candidates could not decide, so
 * they took the dense coarse screen. Writes min(n, 11) values.
 * Errors: EINVAL, EDEVICE.
 */
int hloc_query_info(hloc_db *db, int64_t *out, int32_t n);

/*
 * Region ids chosen for each frame by the last query call (waits for it):
 * nq x n_regions_eff int32, sorted by (distance to representative, id); in
 * id order when every non-empty region was searched. *nq and *n_regions_eff
 * receive the sizes; `out` may be NULL to get only the sizes.
 * Errors: EINVAL, ESTATE, EDEVICE.
 */
int hloc_last_regions(hloc_db *db, int32_t *out, int32_t *nq, int32_t *n_regions_eff);

/*
 * Workspaces: the scratch memory of one batch in flight (frame copies,
 * candidate screen distances, schedule, counters). The calls above use the database's
 * default workspace; a caller that wants several batches in flight at once
 * (on several streams) gives each its own workspace. A workspace belongs to
 * one database and must be freed before it.
 *   hloc_ws_create   new workspace (EINVAL, ENOMEM, EDEVICE).
 *   hloc_ws_free     waits for the device, then releases it (NULL ignored).
 *   hloc_ws_reserve  as hloc_reserve, for this workspace.
 *   hloc_ws_query_async  as hloc_query_batch_async, using this workspace.
 *   hloc_ws_query_info   as hloc_query_info, for this workspace.
 */
int hloc_ws_create(hloc_db *db, hloc_ws **out);
void hloc_ws_free(hloc_ws *ws);
int hloc_ws_reserve(hloc_ws *ws, int32_t nq_max, int32_t nreq_max, int32_t k_max,
                    int32_t n_regions_max);
int hloc_ws_query_async(hloc_ws *ws, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                        const int32_t *req_offsets, int32_t nreq, int32_t precision,
                        int64_t *idx, float *dist, double *xy, int32_t *tile, int32_t *flags,
                        void *stream);
int hloc_ws_query_info(hloc_ws *ws, int64_t *out, int32_t n);

/*
 * Captured batches: hloc_ws_capture records the whole kernel sequence of one
 * batch (arguments as hloc_query_batch_async, all pointers device memory)
 * into a HIP graph held by the workspace, without running it; it sizes the
 * workspace first, so nothing is allocated while recording.
 * hloc_ws_replay(ws, stream) launches that graph on `stream`: the batch runs
 * again on whatever the captured input buffers hold at that time, writing the
 * captured output buffers. The buffers must stay valid while the graph is in
 * use; capturing again replaces the graph. The graph holds the addresses of
 * the workspace's buffers and of the database's arrays: a later call that
 * grows a buffer of this workspace, or hloc_set_regions,
 * hloc_set_aggregation or hloc_set_region_labels on its database, drops or
 * outdates it, and replay then returns ESTATE until the batch is captured
 * again. Errors: EINVAL, ESTATE (replay without a current capture),
 * EUNSUPPORTED, ENOMEM, EDEVICE.
 */
int hloc_ws_capture(hloc_ws *ws, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                    const int32_t *req_offsets, int32_t nreq, int32_t precision, int64_t *idx,
                    float *dist, double *xy, int32_t *tile, int32_t *flags);
int hloc_ws_replay(hloc_ws *ws, void *stream);

/*
 * Device-time profile of the query path, measured with HIP events recorded on
 * the query's stream around each phase:
 *   HLOC_PHASE_PREP      query norms and padded copy
 *   HLOC_PHASE_COARSE    coarse screen against the region representatives
 *   HLOC_PHASE_COARSE_SELECT select + FP64 re-score of the regions of each frame
 *   HLOC_PHASE_SCHED     region -> frames lists and work items
 *   HLOC_PHASE_SCREEN    fine screen of the narrow work items (and of every item
 *                        at padded lengths without a register kernel)
 *   HLOC_PHASE_SCREEN_WIDE fine screen of the wide work items (regions kept by
 *                        more than 16 frames)
 *   HLOC_PHASE_SELECT    per-frame select, FP64 rerank, certificate, exact fallback
 *   HLOC_PHASE_AGGREGATE aggregation of each request
 *   HLOC_PHASE_COARSE_DEFER dense coarse screen and select of the frames the
 *                        fused coarse product's kept candidates could not
 *                        decide (bf16 coarse screens)
 * (kernels of a phase dispatched with start/stop events). It covers the
 * default workspace. hloc_profile(db, 1) clears the record and starts
 * recording for later query calls; hloc_profile(db, 0) stops. hloc_profile_read() waits for the device,
 * writes for each of min(n, HLOC_NUM_PHASES) phases the summed milliseconds
 * and the number of calls recorded, and clears the record.
 * Errors: EINVAL, EDEVICE.
 */
enum {
  HLOC_PHASE_PREP = 0,
  HLOC_PHASE_COARSE = 1,
  HLOC_PHASE_SCHED = 2,
  HLOC_PHASE_SCREEN = 3,
  HLOC_PHASE_SELECT = 4,
  HLOC_PHASE_AGGREGATE = 5,
  HLOC_PHASE_SCREEN_WIDE = 6,
  HLOC_PHASE_COARSE_SELECT = 7,
  HLOC_PHASE_COARSE_DEFER = 8,
  HLOC_NUM_PHASES = 9
};
int hloc_profile(hloc_db *db, int32_t enable);
int hloc_profile_read(hloc_db *db, double *ms, int64_t *calls, int32_t n);

/*
 * Tiles of the fine screen: rows per work item (a multiple of 16, at most 128;
 * regions are cut into chunks of this many rows, at most 64 for regions kept
 * by more than 16 frames) and blocks per compute unit of the persistent screen
 * launches (1 .. 32). They change the speed only: results are the same for
 * every choice. Default 64 and 8.
 *   hloc_set_tiles / hloc_get_tiles   set or read a database's tiles
 *                                     (EINVAL out of range or NULL).
 *   hloc_autotune   times every candidate (rows 32, 64, 96, 128 x blocks 4,
 *                   8, 16) on a sample batch q (device memory, nq frames) with
 *                   the given k, n_regions and precision, `reps` timed runs
 *                   each after one warm-up, keeps the fastest (median time)
 *                   and writes it to *best and its time to *best_ms.
 *                   Allocates scratch outputs. Errors: as hloc_query_batch.
 */
typedef struct {
  int32_t rows_per_item;
  int32_t blocks_per_cu;
} hloc_tiles;
int hloc_set_tiles(hloc_db *db, const hloc_tiles *tiles);
int hloc_get_tiles(hloc_db *db, hloc_tiles *tiles);
int hloc_autotune(hloc_db *db, const float *q, int32_t nq, int32_t k, int32_t n_regions,
                  int32_t precision, int32_t reps, hloc_tiles *best, double *best_ms);

/*
 * Request server: continuous batching of localization requests (the
 * client/server request model of Section 3.1: a request brings the frames
 * around one position, the server returns each frame's top-N candidates and
 * one floor-plan position). Requests of 1 .. max_batch_frames frames are
 * queued as they arrive; whenever one of the server's slots is free, a
 * launcher thread packs the waiting requests, oldest first and never split,
 * into one batch of at most max_batch_frames frames and runs it on that
 * slot's workspace and stream, so up to `slots` batches overlap on the
 * device while new requests keep arriving. A completion thread returns each
 * request's results. A request's results are the same whatever it shares a
 * batch with (every step is per frame or per request).
 *
 * Admission by device memory: each slot holds the workspace and input/output
 * buffers of one full batch, sized once at creation; the server takes
 * min(max_slots, hbm_budget_bytes / bytes per slot) slots (ENOMEM if not even
 * one fits; hbm_budget_bytes = 0 means no limit). Admission of requests: at
 * most max_queue_frames frames wait at once; beyond that submit returns
 * HLOC_EBUSY.
 *
 * While a server exists the database is read-only: hloc_set_regions and
 * hloc_set_aggregation return ESTATE. Frames are copied at submit; results
 * are copied out at wait. Server calls may come from any threads.
 */
typedef struct {
  int32_t k;                /* candidates per frame computed (1 .. HLOC_MAX_K) */
  int32_t n_regions;        /* regions searched per frame (>= 1) */
  int32_t precision;        /* hloc_precision of the screen */
  int32_t max_batch_frames; /* frames per batch (>= 1); also the largest request */
  int32_t max_slots;        /* batches in flight at most (>= 1) */
  int32_t max_queue_frames; /* frames waiting at most (>= max_batch_frames) */
  int64_t hbm_budget_bytes; /* device memory for all slots; 0 = no limit */
} hloc_server_config;

/* Errors: EINVAL (config out of range), ESTATE (no regions), EUNSUPPORTED,
 * ENOMEM (budget below one slot, or allocation failed), EDEVICE. */
int hloc_server_create(hloc_db *db, const hloc_server_config *cfg, hloc_server **out);

/*
 * Queue one request: frames is host nframes x d float32 (copied), nframes in
 * 1 .. cfg.max_batch_frames; k_req in 1 .. cfg.k candidates per frame
 * returned and pooled by the aggregation (nframes x k_req at most
 * HLOC_MAX_REQUEST_CANDIDATES). *ticket identifies it for hloc_server_wait.
 * Errors: EINVAL, EBUSY (queue full), EDEVICE (the server stopped after a
 * device error).
 */
int hloc_server_submit(hloc_server *srv, const float *frames, int32_t nframes, int32_t k_req,
                       uint64_t *ticket);

/*
 * Wait up to timeout_ms (< 0: no limit) for a request and copy its results:
 * idx / dist nframes x k_req (as hloc_query_batch), xy[2], tile[2], flags[1]
 * (any output may be NULL) and latency_ms (submit to completion, may be
 * NULL). A successful wait releases the ticket. Errors: EINVAL (unknown
 * ticket), ETIMEDOUT (the request stays queued or running; wait again),
 * EDEVICE.
 */
int hloc_server_wait(hloc_server *srv, uint64_t ticket, int32_t timeout_ms, int64_t *idx,
                     float *dist, double *xy, int32_t *tile, int32_t *flags, double *latency_ms);

/*
 * Counters: out[0] slots, out[1] bytes of device memory per slot, out[2]
 * batches run, out[3] requests completed, out[4] frames completed, out[5]
 * largest batch (frames), out[6] frames waiting now, out[7] most frames
 * waiting at once, out[8] most batches in flight at once, out[9] submits
 * refused with EBUSY. Writes min(n, 10) values. Errors: EINVAL.
 */
int hloc_server_stats(hloc_server *srv, int64_t *out, int32_t n);

/* Finish the batches in flight, drop queued requests and release the server
 * (NULL is ignored). Must be called before hloc_free_db of its database. */
void hloc_server_free(hloc_server *srv);

/*
 * Omnidirectional feature of 1-D panoramic signals (Section 3: the magnitude
 * of the Fourier transform of the omnidirectional vector, invariant to the
 * camera's heading): for each signal x (len samples around the full circle)
 * out[j] = | sum_t x_t exp(-2 pi i j t / len) |, j = 0 .. d-1, computed in
 * FP64 and rounded once to float32. The rows are ready for hloc_build_db
 * (database) or as query frames.
 *   signals  device, nsig x len float32, row-major (finite values)
 *   nsig     signals (>= 0; 0 does nothing)
 *   len      power of two in 2 .. 2048
 *   d        bins kept, 1 .. len/2 + 1 (higher bins mirror these)
 *   out      device, nsig x d float32, row-major (written)
 *   stream   hipStream_t to enqueue on (NULL: the null stream); runs on the
 *            current HIP device; the call returns once the kernel is enqueued.
 * Needs no database. Errors: EINVAL (sizes out of range, NULL buffers with
 * nsig > 0; checked before any device call), EDEVICE.
 */
int hloc_fft_features_async(const float *signals, int64_t nsig, int32_t len, int32_t d, float *out,
                            void *stream);

/* Release every resource of the database (NULL is ignored). */
void hloc_free_db(hloc_db *db);

/* Message of the last non-OK return on this thread ("" if none). */
const char *hloc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HLOC_H */
