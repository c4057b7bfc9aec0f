/*
 * ccl.h -- C-ABI of the MI355X (gfx950) black-and-white connected-component
 * labeling and analysis library (libccl.so).
 *
 * Operation (Lemaitre & Lacassagne, "A new run-based Connected Component
 * Labeling for efficiently analyzing and processing holes", 2020):
 *   - foreground (nonzero) components under 8-adjacency and background
 *     components under 4-adjacency, found by union of runs of consecutive
 *     rows (Sec. 3.2, B&W unification; Sec. 2, segment detection);
 *   - the label image: every pixel receives the final label of its
 *     component (Sec. 3.2, relabeling);
 *   - per component the bounding box and the raw moments S, Sx, Sy
 *     (Sec. 1; ComputeFeatures and the feature merge of the closure);
 *   - the inclusion (adjacency) tree: the parent of a component is the unique
 *     adjacent component that surrounds it (Sec. 3.1 definitions; obtained
 *     from the initial adjacency of the component's first pixel);
 *   - the Euler number, #foreground components - #holes (Sec. 1, Table 1).
 *
 * Conventions (readings where the paper is silent):
 *   - the image is surrounded by a one-pixel background frame on all four
 *     sides; the background component connected to it is the exterior, id 0;
 *   - every other component (either colour, one id space) is numbered by the
 *     raster rank (row-major) of its first pixel: 1, 2, ...;
 *   - x is the column, y the row; Sx sums x, Sy sums y;
 *   - the exterior may be empty: S = Sx = Sy = 0 and bounding box
 *     (INT32_MAX, -1, INT32_MAX, -1).
 * Results are exact integers and deterministic (independent of scheduling).
 *
 * Memory: every pointer is DEVICE memory unless marked [host].  The caller
 * owns the input, all outputs and the workspace; the library keeps no state
 * between calls.  All calls are asynchronous on `stream` (a hipStream_t,
 * NULL = the null stream) and return once the work is enqueued.
 *
 * Errors: functions return 0 or a negative CCL_E* code; argument errors are
 * detected on the host before anything is enqueued.  Table capacity is
 * checked on the device: when the number of labels exceeds `cap`, the tables
 * receive only the entries with id < cap and counts[0] still holds the true
 * number of labels; the caller compares after synchronising.
 */
#ifndef CCL_H
#define CCL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CCL_OK 0
#define CCL_EINVAL (-1)    /* null pointer, w <= 0, h <= 0, pitch < w, w*h >= 2^31-1, cap < 1 */
#define CCL_ENOSPC (-2)    /* workspace smaller than ccl_workspace_bytes()            */
#define CCL_EHIP (-3)      /* the HIP runtime refused a launch                          */
#define CCL_ECAPACITY (-4) /* (reported by callers) more labels than table capacity    */
#define CCL_ETOOBIG (-5)   /* batch: more than 2^31-1 union-find nodes in one launch    */

/* Per-component features; 40 bytes, 8-byte aligned. */
typedef struct {
  int32_t xmin, xmax, ymin, ymax; /* bounding box, inclusive */
  int64_t S, Sx, Sy;              /* area, sum of x, sum of y */
} ccl_feature_t;

/* Output tables of one image.  Any table pointer may be NULL to skip it
 * (labels == NULL gives the features-only mode: no 4 B/pixel write). */
typedef struct {
  int32_t *labels;          /* [h*w] row-major, row stride w: canonical id per pixel */
  ccl_feature_t *features;  /* [cap] indexed by id */
  int32_t *parent;          /* [cap] parent[0] = -1; parent[c] has the other colour */
  uint8_t *color;           /* [cap] 1 = foreground, 0 = background; color[0] = 0 */
  int64_t cap;              /* [host] table capacity (entries); w*h+1 always suffices */
  int64_t *counts;          /* [2] out: counts[0] = number of labels, counts[1] = Euler number */
} ccl_outputs_t;

/* One image of a batch (host-side description). */
typedef struct {
  const uint8_t *img; /* [h*pitch] bytes, nonzero = foreground */
  int32_t w, h;
  int64_t pitch;      /* row stride in bytes, >= w */
  ccl_outputs_t out;
} ccl_image_t;

/* [host] Workspace bytes needed by ccl_label for a w x h image (pure; 0 on
 * bad input). */
size_t ccl_workspace_bytes(int32_t w, int32_t h);

/* [host] The variant (see below) ccl_label, ccl_label_traced and
 * ccl_label_noalloc run for a w x h image: 16 x 128 tiles up to 1.5
 * Mpixel, 32 x 128 tiles up to 6 Mpixel, else 64 x 128 tiles (smaller
 * images are faster with smaller tiles), with super-tiles of 8 x 8 tiles
 * (variant 9) where the image holds 256 of them or more, else of 4 x 4
 * (variant 0).  Results never depend on it.  CCL_EINVAL for w or h <= 0. */
int32_t ccl_variant_for(int32_t w, int32_t h);

/* Label one image: img[y*pitch + x], y < h, x < w.  Enqueues the whole path
 * on `stream`, in the variant ccl_variant_for(w, h) names.  `ws` needs no
 * initialisation; its contents are scratch. */
int ccl_label(const uint8_t *img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t *out, void *ws,
              size_t ws_bytes, void *stream);

/* Bytes of the per-GPU scratch array of ccl_label_noalloc (96 MiB: images
 * whose ccl_workspace_bytes is at most this, e.g. up to 4096 x 4096). */
#define CCL_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)

/* ccl_label for callers that cannot allocate device memory (code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc): the same work and outputs as ccl_label, with the workspace
 * taken from a static array of CCL_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends.  The caller passes
 * the input and the outputs as for ccl_label; the call allocates nothing.
 * The current device (hipSetDevice) must be the one `stream` runs on; the
 * array's address on that device is looked up on the first call there.
 * Every call on one GPU shares that GPU's array: calls whose work may
 * overlap on the device (other streams, or another host thread) race and
 * give wrong results; calls on one stream are ordered and safe.  The
 * array needs no clearing (every kernel writes the scratch it reads).
 * Errors: CCL_EINVAL as for ccl_label; CCL_ENOSPC when the image needs more
 * workspace than CCL_NOALLOC_SCRATCH_BYTES (ccl_workspace_bytes(w, h)
 * tells); CCL_EHIP when the runtime cannot give the array's address or
 * refuses a launch.  Nothing is enqueued on an argument error. */
int ccl_label_noalloc(const uint8_t *img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t *out,
                      void *stream);

/* ccl_label with the connectivity pair chosen (the note after the
 * unification algorithm, Sec. 3.2): fg_adjacency = 8 is the default pair
 * (8-adjacent foreground, 4-adjacent background); 4 the complementary one
 * (4-adjacent foreground, 8-adjacent background: components, tree and
 * Euler number E = #foreground components - #holes under that pair).  It
 * runs in the 64 x 128 tile shape of variant 0 and needs
 * ccl_workspace_bytes_v(w, h, 0) of workspace; CCL_EINVAL for any other
 * fg_adjacency. */
int ccl_label_conn(const uint8_t *img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t *out, void *ws,
                   size_t ws_bytes, void *stream, int32_t fg_adjacency);

/* Number of HIP events ccl_label_traced records: one before each of the
 * path's nine kernels, in launch order, and one after the last. */
#define CCL_TRACE_EVENTS 10

/* Same work as ccl_label, with `events` [host array of CCL_TRACE_EVENTS
 * hipEvent_t created by the caller] recorded on `stream` around every kernel,
 * so that per-kernel durations can be read with hipEventElapsedTime after the
 * stream completes.  For measurement; no synchronisation is added. */
int ccl_label_traced(const uint8_t *img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t *out, void *ws,
                     size_t ws_bytes, void *stream, void *const *events);

/* [host] Name of kernel k (0..CCL_TRACE_EVENTS-2) in launch order, or NULL. */
const char *ccl_kernel_name(int k);

/* Variants: the path compiled for several tile shapes, workgroup sizes,
 * two ways of summing the partial features of components that cross tiles
 * (an LDS hash table per group of tiles, or direct global atomics) and merge
 * schedules (the side of the super-tiles whose inner seams are merged in LDS
 * before the seams between them are merged in device memory, and the number
 * of tiles per workgroup of the root reduction).  All variants give
 * identical results; they differ in speed per workload.
 * Variant 0 (64 x 128 tiles, 256 threads, LDS hash) is the default for
 * large images; ccl_variant_for names the one a single-image call takes.
 * For tiles of 8192 pixels or more the relabeling kernel
 * (k_tile_emit) always runs 512 threads per tile. */

/* [host] Number of compiled variants. */
int32_t ccl_num_variants(void);

/* [host] Tile rows, tile columns, reduction (1 = LDS hash, 0 = direct
 * atomics), threads per tile workgroup, super-tile side (tiles) and tiles per
 * root-reduction workgroup (1 for direct atomics; the largest group: the
 * default variants of tiles over 4096 pixels take 128 only for a single image
 * of at least 256 such groups, else 64) of `variant` (any output pointer may
 * be NULL); CCL_EINVAL for an unknown index. */
int ccl_variant_info(int32_t variant, int32_t *tile_h, int32_t *tile_w, int32_t *hash_reduce, int32_t *threads,
                     int32_t *super_tile, int32_t *reduce_group);

/* [host] Workspace bytes of `variant` for a w x h image (pure; 0 on bad input). */
size_t ccl_workspace_bytes_v(int32_t w, int32_t h, int32_t variant);

/* ccl_label with an explicit variant. */
int ccl_label_v(const uint8_t *img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t *out, void *ws,
                size_t ws_bytes, void *stream, int32_t variant);

/* Batch: `n` images labeled by one sequence of launches in which every
 * kernel covers every tile of every image (sizes may all differ).
 *
 * Why the batch call takes the host array `imgs` and a `variant` besides the
 * device descriptors: the grid of every kernel is a batch total (tiles,
 * super-tiles, seam work items, scan blocks) that depends on the compiled
 * tile shape of the variant.  Computing it on the host from `imgs` needs no
 * device-to-host copy and no synchronisation, so the call stays asynchronous
 * and can be captured into a hipGraph.  The device block is what the kernels
 * read; it must be the one ccl_batch_prepare wrote for the same `imgs` and
 * `variant`.  Every descriptor carries a digest of the launch shape it was
 * placed for (variant shape and batch totals); kernels of another shape skip
 * it, and the image's counts[0] is set to -1 (nothing else is written).
 *
 * [host] ccl_batch_sizes: bytes of the device descriptor block and of the
 * workspace for the images described in `imgs` [host] under `variant`. */
int ccl_batch_sizes(const ccl_image_t *imgs, int32_t n, int32_t variant, size_t *desc_bytes, size_t *ws_bytes);

/* [host] Write the descriptor block into `host_desc` (desc_bytes from
 * ccl_batch_sizes); the caller copies it to device memory before
 * ccl_label_batch runs and keeps it there while the batch may run again. */
int ccl_batch_prepare(const ccl_image_t *imgs, int32_t n, int32_t variant, void *host_desc, size_t desc_bytes);

/* Enqueue the batch.  `dev_desc` [device] holds the block written by
 * ccl_batch_prepare for the same `imgs` [host] and `variant` (a block placed
 * for other images or another variant is refused image by image on the
 * device: counts[0] = -1).  Capturable in a hipGraph and replayable: it
 * allocates nothing, never synchronises and records no memset (every kernel
 * writes all the scratch it reads). */
int ccl_label_batch(const ccl_image_t *imgs, int32_t n, int32_t variant, const void *dev_desc, void *ws,
                    size_t ws_bytes, void *stream);

/* Hole filling (Sec. 3.2, the transitive closure's optional step in
 * Algorithm 3; Fig. 2, "hole filled"): a component whose surrounding is not
 * the exterior is merged into it, so every hole, with everything nested in
 * it, joins the top-level foreground component around it.  The result is the
 * labeling of the filled image (the complement of the exterior): the exterior
 * (id 0, unchanged) and the top-level foreground components, with canonical
 * ids (raster rank of the first pixel), merged S/Sx/Sy, their own bounding
 * boxes, parent 0, colour 1, and counts = {number of filled labels, Euler
 * number = number of filled foreground components}.
 *
 * `in`: the outputs of ccl_label / ccl_label_batch for a w x h image, on the
 * device (parent and counts required; labels / features when the filled
 * ones are asked for); the number of labels is read from in->counts[0] on
 * the device, so no synchronisation is needed between the two calls.  If
 * that labeling's tables were truncated (counts[0] > cap), out->counts[0] is
 * set to -1 and nothing else is written.
 * `out`: filled labels [w*h] (row stride w), features, parent, colour
 * [out->cap] (each may be NULL) and counts [2]; as for ccl_label, entries
 * with id >= out->cap are dropped while counts[0] stays true.  The number of
 * filled labels never exceeds the number of labels.
 * `map` [in->cap] (device, may be NULL): filled id of every original id.
 * `ws` [ccl_fill_workspace_bytes(in->cap)] scratch, no initialisation.
 * Errors as for ccl_label (CCL_EINVAL, CCL_ENOSPC, CCL_EHIP), on the host. */
size_t ccl_fill_workspace_bytes(int64_t cap);
int ccl_fill_holes(const ccl_outputs_t *in, int32_t w, int32_t h, const ccl_outputs_t *out, int32_t *map, void *ws,
                   size_t ws_bytes, void *stream);

/* Serving: continuous batching over ccl_label_batch.  The paper labels one
 * image at a time; this front end runs the same path for a stream of requests
 * of any sizes.  The calls take a caller-owned device pool (so that the
 * library allocates no device memory and admission is an exact test of a
 * request's footprint against that pool), name requests by a caller tag at
 * submission, and report them through a non-blocking poll that hands back
 * device pointers into the pool, so results stay on the device until the
 * caller releases them.  Requests are admitted in arrival order as soon as a slot and
 * device memory for their whole footprint are free; everything admitted at one
 * poll forms a micro-batch, launched on the next idle one of the server's
 * streams, so that newly admitted work overlaps earlier micro-batches.
 *
 * Memory: `pool` [device, caller-owned, >= 256-byte aligned] is sub-allocated
 * first-fit by the server for every request's input copy, label image and
 * tables and for each micro-batch's descriptors, workspace and counts; the
 * server itself allocates no device memory.  It creates its streams (default
 * priority) and events and grows pinned host staging for descriptors and
 * counts (hipHostMalloc).  A server is used by one host thread at a time;
 * servers are independent of each other.
 *
 * Errors: CCL_EINVAL (bad argument, duplicate or unknown tag, request not
 * done), CCL_ENOSPC (a request's footprint exceeds the whole pool), CCL_EHIP
 * (the HIP runtime failed; the server then returns CCL_EHIP from every call
 * but ccl_server_destroy). */
typedef struct ccl_server ccl_server_t;

typedef struct {
  int32_t max_slots;   /* requests admitted and not yet released, >= 1 */
  int32_t streams;     /* micro-batches in flight at once, 1..16 */
  int32_t max_batch;   /* requests per micro-batch, >= 1 */
  int32_t variant;     /* path variant, 0..ccl_num_variants()-1 */
  int32_t cap_divisor; /* first table capacity of a w x h request:
                          min(w*h+1, max(1024, (w*h+1)/cap_divisor)); >= 1 */
} ccl_server_config_t;

/* A finished request. */
typedef struct {
  int64_t tag;
  int32_t status;    /* CCL_OK; CCL_ENOSPC: the tables this image needs do not fit the pool
                        (n_labels holds the number of labels; no outputs); or the code a batch
                        entry point refused its micro-batch with (no outputs) */
  int32_t w, h;
  int32_t launches;  /* 1, or 2 when the first table capacity was too small and the request ran
                        again with exactly n_labels entries */
  int64_t n_labels, euler;
  ccl_outputs_t out; /* device pointers into the pool, valid until ccl_server_release(tag);
                        out.counts = NULL (the counts are n_labels and euler above) */
} ccl_done_t;

typedef struct {
  int64_t queued;     /* submitted, not yet admitted */
  int64_t live;       /* admitted, not yet released (holding pool memory) */
  int64_t in_flight;  /* micro-batches running */
  int64_t ready;      /* finished, not yet returned by ccl_server_poll */
  int64_t pool_used, pool_bytes;
  int64_t admitted, completed, launches, relaunched;
} ccl_server_stats_t;

/* [host] Create a server over `pool`; `cfg` NULL takes max_slots 256, streams
 * 4, max_batch 64, variant 0, cap_divisor 4. */
int ccl_server_create(void *pool, size_t pool_bytes, const ccl_server_config_t *cfg, ccl_server_t **srv);

/* [host] Pool bytes a w x h request needs when it runs alone (its blocks, one
 * descriptor, its workspace and its counts, each rounded to 256 bytes). */
int ccl_server_footprint(const ccl_server_t *srv, int32_t w, int32_t h, size_t *bytes);

/* [host] Queue a request: `img` [host] h rows of `pitch` bytes; it must stay
 * valid and unchanged until ccl_server_poll reports `tag` (pinned memory
 * makes the upload asynchronous).  `tag` is the caller's name for the request
 * and must not name a request that is still unreleased.  Nothing is enqueued
 * on the device here. */
int ccl_server_submit(ccl_server_t *srv, const uint8_t *img, int32_t w, int32_t h, int64_t pitch, int64_t tag);

/* [host] One scheduling step, never blocking: collect finished micro-batches,
 * admit and launch what fits, then copy up to `max_done` finished requests
 * into `done` [host] in completion order (*n_done of them). */
int ccl_server_poll(ccl_server_t *srv, ccl_done_t *done, int32_t max_done, int32_t *n_done);

/* [host] Give a finished request's pool memory back.  The caller's own work
 * on its outputs must have completed. */
int ccl_server_release(ccl_server_t *srv, int64_t tag);

/* [host] Counters and occupancy. */
int ccl_server_stats(const ccl_server_t *srv, ccl_server_stats_t *st);

/* [host] Wait for the micro-batches in flight, then free the server's streams,
 * events and staging.  The pool stays the caller's. */
int ccl_server_destroy(ccl_server_t *srv);

/* [host] Static message for a CCL_E* code. */
const char *ccl_strerror(int code);

/* [host] Tile shape compiled into this library (rows, columns). */
void ccl_tile_shape(int32_t *tile_h, int32_t *tile_w);

#ifdef __cplusplus
}
#endif
#endif /* CCL_H */
