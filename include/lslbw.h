/*
 * lslbw.h -- C-ABI of the single-thread host (CPU) implementation of the
 * paper's own algorithm, LSL-BW (liblslbw.so), for a like-for-like CPU
 * comparison with the GPU path of ccl.h.
 *
 * Method (Lemaitre & Lacassagne, "A new run-based Connected Component
 * Labeling for efficiently analyzing and processing holes", 2020), one row
 * at a time, one thread:
 *   - segment detection (Sec. 2, Algorithm 1): per-pixel relative labels of
 *     the row (odd = foreground run, even = background run, run 0 background
 *     and possibly empty) and the run boundaries;
 *   - B&W unification (Sec. 3.2, Algorithm 2): every run of the row against
 *     the runs of the row above, foreground runs widened by one pixel on each
 *     side (8-adjacency) and background runs not (4-adjacency), or the other
 *     way round for the complementary pair; union by minimum in the
 *     equivalence table; features per run; a new label records the label of
 *     the run on its left as its initial adjacency; the first and last
 *     background runs of every row are attached to the exterior (label 0);
 *   - transitive closure (Sec. 3.2, Algorithm 3): one forward pass over the
 *     labels that points every label at its root, merges features into the
 *     roots and points the initial adjacency of every root at its root (the
 *     adjacency tree, Sec. 3.1); optionally hole filling;
 *   - relabeling (Sec. 3.2, Algorithm 4): every run of every row receives its
 *     final label.
 *
 * Readings where the paper is silent (the same as the GPU path's, so that
 * both produce identical outputs):
 *   - the row above row 0 is a virtual background row that belongs to the
 *     exterior (label 0);
 *   - the image has a one-pixel background frame on all four sides: besides
 *     the first and last background runs of every row, every background run
 *     of the last row is attached to the exterior;
 *   - the initial adjacency of a new label on a row's first run is the
 *     exterior; the closure leaves label 0 alone (its parent is -1);
 *   - final numbering: roots compacted in increasing order (the exterior is
 *     0, every other component gets the raster rank of its first pixel,
 *     since labels are created in raster order and a root is its
 *     component's first run);
 *   - Euler number = #foreground components - #holes (holes: every
 *     background component but the exterior);
 *   - hole filling: the closure's test merges every root whose surrounding
 *     is not the exterior into that surrounding; the outputs are then the
 *     filled labeling (exterior plus top-level foreground components, parent
 *     0, merged S / Sx / Sy, Euler number = their count).
 *
 * Memory: every pointer is HOST memory.  The caller owns the image and all
 * outputs; a context owns the working tables (equivalences, initial
 * adjacency, features per provisional label, runs of every row), allocated
 * by lslbw_create and grown when an image needs more labels.  A context is
 * used by one thread at a time.
 *
 * Errors: 0 or a negative LSLBW_E* code; nothing is written on an argument
 * error.  Tables hold the entries with id < cap; counts[0] is always the true
 * number of labels.
 */
#ifndef LSLBW_H
#define LSLBW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LSLBW_OK 0
#define LSLBW_EINVAL (-1) /* null context / image / counts, pitch < w, size other than the context's */
#define LSLBW_ENOMEM (-2) /* a working table could not be allocated or grown */

/* What a call computes besides the B&W labels and the adjacency tree (the
 * paper's base configuration, "BWA"). */
#define LSLBW_FEATURES 1 /* bounding box, S, Sx, Sy per component ("F") */
#define LSLBW_RELABEL 2  /* the label image ("R") */
#define LSLBW_EULER 4    /* the Euler number into counts[1] ("E"; else counts[1] = 0) */
#define LSLBW_FILL 8     /* hole filling in the closure */
#define LSLBW_FG4 16     /* complementary pair: 4-adjacent foreground, 8-adjacent background */

/* Per-component features, 40 bytes: bounding box (inclusive), area, sum of x
 * (column), sum of y (row). */
typedef struct {
  int32_t xmin, xmax, ymin, ymax;
  int64_t S, Sx, Sy;
} lslbw_feature_t;

/* Duration of the last call: time-stamp-counter ticks (the TSC runs at the
 * processor's nominal clock, so ticks / pixels is the paper's cycles per
 * pixel) and nanoseconds of a monotonic clock. */
typedef struct {
  uint64_t tsc;
  uint64_t ns;
} lslbw_time_t;

typedef struct lslbw_ctx lslbw_ctx_t;

/* Working tables for w x h images (w, h >= 1, w*h < 2^31).  The equivalence
 * tables start at room for w*h/4 + w + 2 labels and double when needed. */
int lslbw_create(int32_t w, int32_t h, lslbw_ctx_t **ctx);
void lslbw_destroy(lslbw_ctx_t *ctx);

/* Label img[y*pitch + x] (nonzero = foreground), x < w, y < h, of the
 * context's size.  Outputs (any of the table pointers may be NULL; labels and
 * feat are only written when RELABEL / FEATURES are asked for):
 *   labels [w*h] row stride w, canonical id per pixel;
 *   feat, parent, color [cap] indexed by canonical id (parent[0] = -1,
 *     color 1 = foreground);
 *   counts [2]: number of labels, Euler number.
 * `t` (may be NULL) receives the duration of the whole call. */
int lslbw_label(lslbw_ctx_t *ctx, const uint8_t *img, int64_t pitch, int32_t flags, int32_t *labels,
                lslbw_feature_t *feat, int32_t *parent, uint8_t *color, int64_t cap, int64_t *counts,
                lslbw_time_t *t);

#ifdef __cplusplus
}
#endif
#endif /* LSLBW_H */
