/*
 * obg.h -- octree background modelling on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the GPU library libobg.so.  The method is the one of "Background
 * Modeling Using Octree Color Quantization" (arXiv 1412.1945):
 *
 *   1. every pixel colour is a path in an octree: at level i the child index
 *      is built from bit 7-i of R, G and B (Algorithm 1, Store Color);
 *   2. a frame's octree, pruned to depth d (Section 2), is exactly the set of
 *      depth-d paths that occur in the frame; here it is an occupancy bitset;
 *   3. the trees of T training frames are merged, keeping a path when the
 *      fraction of trees that contain it reaches a threshold (Algorithm 2,
 *      Merge Trees, Section 3);
 *   4. a pixel of an incoming frame is foreground when its path is missing
 *      from the merged tree (Algorithm 3, Check Color, Section 4);
 *   5. optionally the frame is split into rectangular regions, each with its
 *      own trees (Sections 3 and 4).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Child index at level i (i = 0 just below the root): 4*r + 2*g + b, where r,
 * g, b are bit 7-i of the 8-bit R, G, B values (the paper prints the index as
 * a sum of the three bits; a sum cannot address eight children, so the bits
 * are concatenated, red most significant).
 * Path key of a depth-d node: its child indices c_0..c_{d-1} as base-8
 * digits, c_0 most significant; 0 <= key < 8^d.
 * Bitset of one tree: ceil(8^d / 32) uint32 words; key k is bit (k & 31) of
 * word (k >> 5).  Bits past 8^d (d = 1) are ignored on input, 0 on output.
 * Regions: region_w = region_h = 0 means one tree per frame.  Otherwise the
 * frame is cut into a row-major grid of region_w x region_h rectangles (the
 * last column/row may be narrower/shorter); region id of pixel (x, y) =
 * (y / region_h) * ceil(width / region_w) + x / region_w.  Per frame the
 * bitsets of all regions are stored back to back, region 0 first.
 * Frames: packed RGB8, pixel x of row y at byte y*row_pitch + 3x (R, G, B);
 * frame f starts frame_pitch bytes after frame f-1.  The buffer must span
 * n_frames * frame_pitch bytes.
 * Masks: per frame height rows of ceil(width / 64) uint64 words; pixel x is
 * bit (x & 63) of word (x >> 6); 1 = foreground; bits past width are 0.
 * Frames follow each other without gaps.
 *
 * Memory and streams: every buffer pointer is a DEVICE pointer owned by the
 * caller.  Calls validate their arguments, enqueue kernels on `stream`
 * (NULL = the default stream) and return without waiting; the library keeps
 * no pointer after a call returns.
 * Outputs are written completely by the call (no pre-zeroing needed).
 * Faults inside a kernel surface at the caller's next synchronisation.
 *
 * Errors: 0 (OBG_OK) or a negative code; obg_last_error() returns a message
 * for the calling thread's last failed call.  Nothing is enqueued when a call
 * fails validation.
 */
#ifndef OBG_H
#define OBG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OBG_OK           0
#define OBG_EINVAL      -1   /* bad size, depth, threshold, NULL pointer ... */
#define OBG_EALIGN      -2   /* frame pointer or pitch not 16-byte aligned    */
#define OBG_EHIP        -3   /* HIP launch / runtime failure                  */
#define OBG_ENOMEM      -4   /* host or device allocation failed              */

typedef struct obg_geom {
    int32_t width, height;     /* pixels, >= 1                                */
    int64_t row_pitch;         /* bytes, >= 3*width, multiple of 16           */
    int64_t frame_pitch;       /* bytes, >= height*row_pitch, multiple of 16  */
    int32_t depth;             /* d in [1, 8]: octree levels kept (Section 2) */
    int32_t region_w, region_h;/* 0,0 = one tree per frame; else >= 1 each    */
} obg_geom;

/* Number of regions of the geometry (1 without regions); -1 if invalid. */
int64_t obg_num_regions(const obg_geom *g);
/* uint32 words of one frame's occupancy: n_regions * ceil(8^d / 32). */
int64_t obg_occ_words(const obg_geom *g);
/* uint64 words of one frame's mask: height * ceil(width / 64). */
int64_t obg_mask_words(const obg_geom *g);

/*
 * Per-frame pruned octrees (Algorithm 1 for every pixel, pruned to depth d
 * as in Section 2), as occupancy bitsets.
 *   rgb    : n_frames frames (layout above), 16-byte aligned.
 *   occ    : out, [n_frames][n_regions][ceil(8^d/32)] uint32; bit k set iff
 *            some pixel of that frame and region has path key k.
 *   counts : out, NULLABLE, [n_frames][n_regions][8^d] uint32; pixels per key
 *            (node pixel counts of the pruned tree; diagnostic).
 * n_frames = 0 enqueues nothing.
 */
int obg_train_frame(const obg_geom *g, const uint8_t *rgb, int32_t n_frames,
                    uint32_t *occ, uint32_t *counts, hipStream_t stream);

/*
 * Merge of per-frame trees (Algorithm 2).  A path key k of region r is kept
 * iff C = number of trees in the window whose bitset has k satisfies
 * C * thr_den >= thr_num * n_trees (the paper compares the fraction of trees
 * holding the path with the threshold; here the comparison is exact in
 * integers).  Because every tree that holds a
 * path also holds all its prefixes, this per-key test gives the same depth-d
 * nodes as the paper's level-by-level recursion.
 *   occ_ring : [ring_len][n_regions][ceil(8^d/32)] uint32, per-frame bitsets.
 *   window   : slots first, first+1, ..., first+n_trees-1 (mod ring_len).
 *   leafset  : out, [n_regions][ceil(8^d/32)] uint32, the merged tree's
 *              depth-d nodes.
 * EINVAL: n_trees < 1, n_trees > ring_len, n_trees > 65535, first outside
 * [0, ring_len), thr_num = 0 (a zero threshold would keep paths no tree
 * has), thr_den = 0.  thr_num > thr_den is allowed: nothing is kept.
 * Only depth and regions of g are used.
 */
int obg_merge(const obg_geom *g, const uint32_t *occ_ring, int32_t ring_len,
              int32_t first, int32_t n_trees, uint32_t thr_num, uint32_t thr_den,
              uint32_t *leafset, hipStream_t stream);

/*
 * Merge of trees built from groups of frames (Section 3 allows one tree per
 * frame or per group of frames).  The window's n_trees slots are taken in
 * groups of `group` consecutive slots, the last group possibly shorter; a
 * group's tree holds every colour of its frames, so its bitset is the OR of
 * the group's bitsets.  Key k is kept iff G * thr_den >= thr_num * n_groups,
 * G = number of groups holding k, n_groups = ceil(n_trees / group).
 * group = 1 is obg_merge.  Arguments and errors as obg_merge, and EINVAL for
 * group < 1.
 */
int obg_merge_groups(const obg_geom *g, const uint32_t *occ_ring, int32_t ring_len, int32_t first,
                     int32_t n_trees, int32_t group, uint32_t thr_num, uint32_t thr_den, uint32_t *leafset,
                     hipStream_t stream);

/*
 * Foreground detection (Algorithm 3 for every pixel, Section 4): mask bit 1
 * iff the pixel's depth-d path key is not in its region's leaf set.
 *   rgb     : n_frames frames (layout above), 16-byte aligned.
 *   leafset : [n_regions][ceil(8^d/32)] uint32 (as written by obg_merge).
 *   mask    : out, [n_frames][height][ceil(width/64)] uint64.
 *   occ_out : out, NULLABLE; when given, the occupancy of every classified
 *             frame as obg_train_frame would write it (one pass over the
 *             pixels produces both; used to keep a ring of recent trees).
 */
int obg_classify(const obg_geom *g, const uint8_t *rgb, int32_t n_frames,
                 const uint32_t *leafset, uint64_t *mask, uint32_t *occ_out,
                 hipStream_t stream);

/*
 * Redraw (Section 2): every frame redrawn with its own pruned octree.  The
 * colour of a depth-d node is its path bits with the remaining 8-d bits zero,
 * and a frame's tree holds every pixel's node, so each channel keeps its top
 * d bits: out byte = rgb byte & (0xFF << (8 - d)).
 *   rgb, out : n_frames frames in the layout above (the same geometry),
 *              16-byte aligned; out may be rgb itself (in place) but must not
 *              otherwise overlap it.  Row padding of out is not written.
 * Regions do not change the result (a pixel's colour is in its region's tree).
 * n_frames = 0 enqueues nothing.
 */
int obg_quantize(const obg_geom *g, const uint8_t *rgb, int32_t n_frames, uint8_t *out, hipStream_t stream);

/*
 * Agreement of foreground masks with ground-truth masks, for the figures of
 * Section 5 (F0 of the background class: P0 = Tn / (Tn + Fn), R0 = Tn /
 * (Tn + Fp), F0 = 2 P0 R0 / (P0 + R0)).
 *   mask, truth : [n_frames][height][ceil(width/64)] uint64 each, the mask
 *                 layout (1 = foreground); bits past width are ignored.
 *   counts      : out, device, 3 uint64: true positives, false positives,
 *                 false negatives over all frames (overwritten).  True
 *                 negatives = n_frames * width * height minus the three.
 * Only width and height of g are used.  n_frames = 0 writes zeros.
 */
int obg_score(const obg_geom *g, const uint64_t *mask, const uint64_t *truth, int32_t n_frames, uint64_t *counts,
              hipStream_t stream);

/*
 * Batched form (Algorithms 1-3 over many streams): many independent camera
 * streams of uneven resolution, depth, training length and threshold in one
 * persistent launch per step.
 *
 * A plan is made once from host descriptions of its streams (geometry,
 * depth, threshold, most frames per run).  Each run then takes a DEVICE
 * array of work items, one per stream that takes part, giving that run's
 * frames, frame counts and output buffers, so one plan serves new frames,
 * new buffers and changing counts without being made again.  A run enqueues
 * on `stream`:
 *   a prepare kernel (one workgroup) that checks the items, writes each
 *   item's status, and lays out the run's work in the plan's device memory;
 *   then the three steps, each ONE persistent launch over all streams (or one
 *   per depth present, when the autotuner picked that):
 *     trees of every training frame (Algorithm 1 with the pruning of
 *     Section 2), the merge of every stream that trained (Algorithm 2, the
 *     stream's threshold), the masks of every test frame (Algorithm 3).
 *   The steps read their item counts from device memory, so they are
 *   captured once in a HIP graph when the plan is made and replayed by every
 *   run (OBG_TUNE_BATCH_GRAPH = 2 launches them directly instead).
 * Per stream, the outputs are byte-identical to the one-stream calls:
 * obg_train_frame over the item's n_train frames, obg_merge of all of them
 * (window = the n_train trees), and obg_classify of its n_test frames.
 *
 * Plan streams: plain geometry (region_w = region_h = 0), depth 1..6,
 * pitches as for the one-stream calls, thr_num, thr_den >= 1,
 * 0 <= max_train <= 65535, max_test >= 0; at most 8192 streams.
 * Work item (device memory, written back only in `status`):
 *   stream    index of a plan stream; each stream at most once per run
 *   n_train   0..max_train training frames at train_rgb (the stream's
 *             frame_pitch apart, 16-byte aligned): their trees are written
 *             to occ [n_train][ceil(8^d/32)] uint32 and their merge to
 *             leafset [ceil(8^d/32)] uint32.  n_train = 0: no trees, and
 *             leafset is the model the test frames are checked against
 *   n_test    0..max_test test frames at test_rgb: masks to mask
 *             [n_test][height][ceil(width/64)] uint64
 *   status    set by the run: OBG_ITEM_OK, or why the item was skipped
 *             (nothing of a skipped item is written)
 * A stream that no item names is left alone.  n_items must be in
 * [0, n_streams] (EINVAL otherwise); n_items = 0 enqueues nothing.  The
 * library reads the item array on the device during the run: it must stay
 * valid until the run completes.  Runs of one plan must not overlap (they
 * share the plan's device memory): issue them on one stream, or order them.
 *
 * obg_plan_tune times launch shapes (one launch per phase or per depth;
 * workgroup size, workgroups per CU, work-item size and dealing of each
 * step) on the given work, which it runs several times, waiting for each;
 * every shape must give the same output bytes (else OBG_EHIP); the plan
 * keeps the fastest and captures its graph again.  It must not overlap a
 * run of the plan.
 */
typedef struct obg_plan_stream {
    obg_geom geom;
    uint32_t thr_num, thr_den;
    int32_t max_train, max_test;
} obg_plan_stream;

typedef struct obg_work_item {
    int32_t stream;
    int32_t n_train, n_test;
    int32_t status;
    const uint8_t *train_rgb;
    const uint8_t *test_rgb;
    uint32_t *occ;
    uint32_t *leafset;
    uint64_t *mask;
} obg_work_item;

#define OBG_ITEM_OK          0
#define OBG_ITEM_BAD_STREAM  1   /* stream outside the plan                     */
#define OBG_ITEM_BAD_COUNT   2   /* n_train or n_test outside [0, max]          */
#define OBG_ITEM_NULL        3   /* a buffer the counts need is NULL            */
#define OBG_ITEM_ALIGN       4   /* frames not 16-, trees 4-, masks 8-aligned   */
#define OBG_ITEM_DUPLICATE   5   /* an earlier item of the run names the stream */

typedef struct obg_plan obg_plan;

typedef struct obg_plan_info {
    int32_t n_streams;
    int64_t max_train_items, max_classify_items;   /* work items of each step at the maxima */
    int32_t train_block, train_wg_per_cu, train_items_per_wg;
    int32_t classify_block, classify_wg_per_cu, classify_span;
    int32_t classify_round_robin;             /* 1: classify items dealt round-robin */
    int32_t per_depth_launches;               /* 1: one launch per depth and phase */
    int32_t graph;                            /* 1: runs replay a graph    */
    int32_t tune_candidates;                  /* shapes timed (obg_plan_tune) */
    double tune_default_ms, tune_best_ms;     /* one run, first vs chosen shape */
} obg_plan_info;

int obg_plan_create(const obg_plan_stream *streams, int32_t n_streams, obg_plan **out);
int obg_plan_tune(obg_plan *plan, const obg_work_item *work_items_dev, int32_t n_items, hipStream_t stream);
int obg_batch_run(obg_plan *plan, const obg_work_item *work_items_dev, int32_t n_items, hipStream_t stream);
int obg_plan_info_get(const obg_plan *plan, obg_plan_info *out);
void obg_plan_destroy(obg_plan *plan);

/*
 * Batched run without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The same work and outputs as obg_plan_create(streams,
 * n_streams) followed by obg_batch_run(plan, work_items_dev, n_items,
 * stream), with the plan's starting launch shape and no graph, but no plan:
 * the per-stream descriptors and the launches' item counts live in a static
 * device array of the library (room for OBG_NOALLOC_MAX_STREAMS streams, each
 * GPU holding its own copy until the process ends).  No device memory is
 * allocated or freed; the descriptors are copied from host memory with
 * hipMemcpyAsync on `stream`.
 *   streams          host array, as for obg_plan_create (read during the call)
 *   n_streams        1..OBG_NOALLOC_MAX_STREAMS (EINVAL otherwise)
 *   work_items_dev   as for obg_batch_run (n_items in [0, n_streams]; each
 *                    item's status is written)
 * Every call on one GPU uses that GPU's array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different HIP streams, or from
 * several threads) race; issue them on one stream or order them.
 * Errors as obg_plan_create and obg_batch_run; nothing is enqueued when
 * validation fails.
 */
#define OBG_NOALLOC_MAX_STREAMS 256
int obg_batch_run_noalloc(const obg_plan_stream *streams, int32_t n_streams, const obg_work_item *work_items_dev,
                          int32_t n_items, hipStream_t stream);

/*
 * Serving: continuous batching of frames that arrive from many cameras.
 *
 * obg_serve_run drives one run to completion.  Frame f of stream s arrives
 * at arrivals[s][f] simulated seconds (finite; a frame that arrives before
 * its predecessor waits for it, so each stream is served in frame order, and
 * its latency counts from its own arrival); simulated time
 * runs `speed` times faster than wall time.  The loop admits arrived frames
 * as long as the HBM budget (one arena: every stream's ring and leaf set,
 * plus the buffers of the frames in flight) allows, forms a batch from the
 * frames of many streams and enqueues it on one of `max_inflight` HIP
 * streams, so that batches overlap on the device while new frames keep
 * arriving.  A batch is: the ingest callback (writes the frames' pixels),
 * the trees of training frames into ring slots, one pass over test frames
 * that writes each mask and each frame's tree, and the merges that are due.
 *   Frames 0 .. n_train-1 of a stream are training frames; after the last
 *   one the model is the merge of all of them (Algorithm 2).  Frame f >=
 *   n_train is test frame t = f - n_train; after every `remerge_period`-th
 *   test frame the model becomes the merge of the last `remerge_window`
 *   frames' trees (same threshold), used from the next frame on (a reading
 *   of the tree update that the paper names but does not define).
 *   Per stream, results do not depend on what else is in the mix.
 * Latency of a test frame = time its mask is complete in HBM minus its
 * arrival (wall clock).  Outputs for checking: per-frame mask checksums
 * (a 64-bit hash of the mask words, `checksums[s * checksum_stride + f]`,
 * NULL = off) and the full masks of the test frames of `watch_streams` copied
 * to host buffers (watch_masks[w], [watch_max_frames][height][ceil(width/64)]).
 * Streams: depth 1..6, one tree per frame or per region (Sections 3 and 4);
 * pixels are packed RGB8 with row pitch 3*width rounded up to 16 bytes.
 * Frames of streams without regions go through one launch per batch.  For a
 * stream with regions, each run of its test (or training) frames in a batch
 * is one pass of the region kernels over per-frame pointer lists (the same
 * results as obg_classify with occ_out, or obg_train_frame, frame by frame),
 * on the batch's HIP stream; geometries only the per-pixel kernel takes go
 * frame by frame through those entry points.  Their merges are obg_merge
 * calls.
 * Admission: a frame takes one arena block (its pixels, and for a test frame
 * its mask).  When a frame does not fit, its stream goes first and no other
 * frame is admitted until it does, so no stream starves; a frame that cannot
 * fit even with nothing in flight ends the run with OBG_ENOMEM.  The library
 * allocates the arena, its slots' staging buffers and streams at the start of
 * the run and frees them before returning.
 * Errors: OBG_EINVAL (bad configuration), OBG_ENOMEM (budget or allocation),
 * OBG_EHIP (a launch or a batch failed, or the scheduler stopped making
 * progress).  Statistics are filled in either way.
 */
typedef struct obg_ingest_item {
    int32_t stream;
    int32_t frame;
    uint8_t *dst;        /* device buffer of height * row_pitch bytes */
} obg_ingest_item;

/* Enqueue the writing of the items' pixels on `stream`; 0 = success. */
typedef int (*obg_ingest_fn)(void *ctx, const obg_ingest_item *items, int32_t n, hipStream_t stream);

typedef struct obg_serve_stream {
    int32_t width, height, depth;
    int32_t n_train;
    uint32_t thr_num, thr_den;
    int32_t region_w, region_h;   /* 0, 0 = one tree per frame; else regions as above */
} obg_serve_stream;

typedef struct obg_serve_config {
    const obg_serve_stream *streams;
    int32_t n_streams;
    const double *const *arrivals;     /* [n_streams][n_arrivals[s]] simulated seconds */
    const int32_t *n_arrivals;
    double speed;                      /* simulated seconds per wall second, > 0 */
    uint64_t budget_bytes;
    int32_t max_inflight;              /* 1..16 batches on the device at once */
    int32_t max_batch_frames;          /* 1..4096 */
    int32_t remerge_period, remerge_window;   /* 1 <= window <= period */
    obg_ingest_fn ingest;
    void *ingest_ctx;
    uint64_t *checksums;               /* NULLABLE */
    int32_t checksum_stride;
    const int32_t *watch_streams;      /* NULLABLE */
    int32_t n_watch;
    uint64_t *const *watch_masks;
    int32_t watch_max_frames;
    /* Checkpoint, NULLABLE (host buffers of obg_serve_state_bytes bytes).
       state_out receives, when the run ends, every stream's merged leaf set,
       its ring of per-frame trees and the index of its next frame (region
       streams and streams of depth 5 or 6 may hold their bitsets in the
       kernels' own bit order, which the stream's record names: a state is
       for restoring, not for reading;
       a state restored under an OBG_TUNE_LAYOUT setting that picks the other
       order for a stream is refused with OBG_EINVAL).  state_in
       restores such a state (written for the same streams: geometry, depth,
       n_train, regions, and the same remerge_window) before the first frame
       is admitted; arrivals[s][i] is then frame next_frame[s] + i, and every
       result of the resumed run equals that of one run over all the frames.
       A state that does not match is refused with OBG_EINVAL. */
    const void *state_in;
    void *state_out;
} obg_serve_config;

typedef struct obg_serve_stats {
    int64_t frames_arrived, frames_served, train_frames, test_frames, pixels;
    int64_t batches, merges, admission_waits;
    double wall_s;
    double lat_p50_ms, lat_p99_ms, lat_max_ms, lat_mean_ms;
    double peak_bytes;                 /* arena bytes in use at the peak */
    int64_t train_pixels, test_pixels;
    /* seconds during which at least one batch was on the device: from its
       first copy to its completion (busy_s), and only its path kernels, from
       the end of ingest to the end of its merges (path_busy_s); overlapping
       batches count once */
    double busy_s, path_busy_s;
} obg_serve_stats;

int obg_serve_run(const obg_serve_config *cfg, obg_serve_stats *stats);
/* Bytes of a serving checkpoint of these streams (-1 if a description is
   invalid): a 16-byte header (magic, n_streams, remerge_window), 48 bytes per
   stream (geometry, ring length, bit order, next frame, tree bytes), then per stream its
   leaf set and its ring of trees, each padded to 8 bytes. */
int64_t obg_serve_state_bytes(const obg_serve_stream *streams, int32_t n_streams, int32_t remerge_window);

/*
 * Launch-shape knobs of the pixel kernels and batches, process-wide, for the
 * autotuner (0 restores the built-in default).  They change speed only:
 * every setting gives the same bytes.
 *   OBG_TUNE_TRAIN_BLOCK        threads per workgroup of occupancy-only
 *                               passes: 256 or 1024 (default 1024; 256 for
 *                               region work items of fewer than 2048
 *                               16-pixel groups)
 *   OBG_TUNE_OCC_BLIND          1 = set occupancy bits with an unconditional
 *                               LDS atomic OR (default for occupancy-only
 *                               passes with regions and for batched trees at
 *                               d = 6), 2 = read the word first and OR only a
 *                               clear bit (default otherwise: fewer colliding
 *                               atomics when many pixels share a key); the
 *                               fused pass always reads first
 *   OBG_TUNE_OCC_WG_PER_CU      workgroups per CU of passes that build
 *                               occupancy (default 2 at 1024 threads, else 4)
 *   OBG_TUNE_CLASSIFY_WG_PER_CU workgroups per CU of classify-only passes
 *                               (default 2, fewer if LDS does not allow)
 *   OBG_TUNE_CLASSIFY_SPAN      16-pixel groups per work item of classify-only
 *                               passes (default 832; 1024 with compact
 *                               tables: d = 6 and most region tables)
 *   OBG_TUNE_CLASSIFY_BLOCK     threads per workgroup of classify passes:
 *                               256 or 512 (default; 256 for fused region
 *                               work items of fewer than 2048 groups)
 *   OBG_TUNE_LAYOUT             LDS order of d <= 5 trees: 1 = wide table
 *                               indexed by the pixel's R,G bytes (default),
 *                               2 = compact
 *   OBG_TUNE_INTERLEAVE         1 = work items dealt round-robin to the
 *                               workgroups, 2 = contiguous runs (default:
 *                               round-robin for classify without regions)
 *   OBG_TUNE_MASK_STAGE         1 = gather a work item's mask in LDS and write
 *                               it in one run (items of <= 1024 groups;
 *                               default), 2 = write each 64-pixel word directly
 *   OBG_TUNE_REGION_CHUNKS      1 = with regions, cut rows of regions into
 *                               chunks of whole region columns when a call
 *                               has too few rows of regions to fill the chip,
 *                               and give passes that build occupancy one work
 *                               item per (frame, chunk) whose words are
 *                               stored (default); 2 = chunks only where a
 *                               row's tables do not fit in LDS
 *   OBG_TUNE_BATCH_PER_DEPTH    shape a plan starts from (obg_plan_create,
 *                               before any tuning, and obg_batch_run_noalloc):
 *                               1 = one persistent launch per phase, 2 = one
 *                               launch per depth present and phase (default)
 *   OBG_TUNE_BATCH_GRAPH        1 = plans capture their steps in a HIP graph
 *                               (default), 2 = runs launch them directly
 *   OBG_TUNE_FUSED_SPAN         16-pixel groups per work item of the fused
 *                               classify + occupancy pass without regions
 *                               (default 4096; items of at most 4096 groups
 *                               gather their masks in LDS)
 */
#define OBG_TUNE_TRAIN_BLOCK         0
#define OBG_TUNE_OCC_BLIND           1
#define OBG_TUNE_OCC_WG_PER_CU       2
#define OBG_TUNE_CLASSIFY_WG_PER_CU  3
#define OBG_TUNE_CLASSIFY_SPAN       4
#define OBG_TUNE_CLASSIFY_BLOCK      5
#define OBG_TUNE_LAYOUT              6
#define OBG_TUNE_INTERLEAVE          7
#define OBG_TUNE_MASK_STAGE          8
#define OBG_TUNE_REGION_CHUNKS       9
#define OBG_TUNE_BATCH_PER_DEPTH     10
#define OBG_TUNE_BATCH_GRAPH         11
#define OBG_TUNE_FUSED_SPAN          12
#define OBG_TUNE_COUNT               13
int obg_tune_set(int key, int value);
int obg_tune_get(int key);   /* current value, 0 = default, -1 = bad key */

/*
 * Measurement probes (not part of the method): streaming kernels that show
 * what the memory system delivers for the pixel kernels' access pattern.
 *   OBG_PROBE_READ       read `bytes` of src in 48-byte steps per lane
 *                        (whole 24 KiB items only); sink gets grid*512 words
 *   OBG_PROBE_READ_WRITE the same reads plus 1/24 as many bytes written to
 *                        dst in one run per item (the classify output ratio)
 *   OBG_PROBE_COPY       copy `bytes` (multiple of 16) from src to dst
 * Pointers are device pointers, 16-byte aligned; dst must hold bytes/24
 * (READ_WRITE) or bytes (COPY); sink must hold grid*512 uint32 (READ*).
 * grid: workgroups of the READ* kernels, 1..65536.
 */
#define OBG_PROBE_READ        1
#define OBG_PROBE_READ_WRITE  2
#define OBG_PROBE_COPY        3
int obg_probe(int kind, const void *src, void *dst, int64_t bytes, uint32_t *sink, int32_t grid,
              hipStream_t stream);

/*
 * Shaped probe (measurement, not part of the method): the READ and
 * READ_WRITE probes above with their launch shape given, so that the
 * ceiling of the classify access pattern can be swept.
 *   kind         OBG_PROBE_READ or OBG_PROBE_READ_WRITE
 *   grid         workgroups, 1..65536
 *   block        threads per workgroup: 256, 512 or 1024
 *   inflight     48-byte groups each lane loads before it uses any: 1, 2, 4
 *   span         groups per item (a multiple of 4 in 4..4096); items are
 *                dealt round-robin over the workgroups; READ_WRITE writes
 *                each item's 2 bytes per group as one run (1/24 of the bytes
 *                read) after the item
 *   phase_items  READ_WRITE only.  0: as above.  n > 0: every workgroup
 *                reads n items (their output staged on chip, n * span * 2
 *                bytes <= 64 KiB), then waits at a grid-wide counter until
 *                every workgroup has read its n items, then writes them, so
 *                that the chip's reads and writes are separated in time.  The
 *                wait is bounded (a workgroup that waited too long goes on);
 *                the launch is cooperative and fails with OBG_EHIP when the
 *                grid cannot be resident at once.
 * sink must hold grid * block + 1 uint32 (the last word is the phased
 * probe's counter, cleared by the call); dst as for OBG_PROBE_READ_WRITE.
 */
typedef struct obg_probe_shape {
    int32_t kind, grid, block, inflight, span, phase_items;
} obg_probe_shape;
int obg_probe_shaped(const obg_probe_shape *shape, const void *src, void *dst, int64_t bytes, uint32_t *sink,
                     hipStream_t stream);

/* Message of the calling thread's last failed call ("" if none). */
const char *obg_last_error(void);

/* Library version string. */
const char *obg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OBG_H */
