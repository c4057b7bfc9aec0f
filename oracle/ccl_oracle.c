/*
 * ccl_oracle.c -- plain, slow, single-threaded CPU oracle for black-and-white
 * connected-component labeling with features, Euler number and inclusion tree.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this file's library.  The HIP product path
 * never links, imports or calls it, and it shares no code, header, table or
 * helper with the HIP path.
 *
 * What it computes (Lemaitre & Lacassagne, "A new run-based Connected
 * Component Labeling for efficiently analyzing and processing holes", 2020):
 *   - foreground (nonzero) components under 8-adjacency and background
 *     components under 4-adjacency (Sec. 3.2, the B&W unification and the note
 *     on the connectivity pair that follows the algorithms);
 *   - per component the bounding box and the raw moments S, Sx, Sy
 *     (Sec. 1 and the ComputeFeatures step of the unification algorithm);
 *   - the Euler number (Sec. 1, Table 1);
 *   - the adjacency / inclusion tree: for each component the unique adjacent
 *     component that surrounds it (definitions in Sec. 3.1).
 *
 * The method reaches these results exactly (integer arithmetic), so this
 * oracle is their plain definition written out, not the paper's run-based
 * algorithm:
 *   1. a disjoint-set forest over one node per pixel plus node 0, the 1-pixel
 *      background frame around the image ("the exterior of the image");
 *      union by minimum index, path halving; one raster pass linking each
 *      pixel with its already-visited neighbours of the same colour
 *      (W, NW, N, NE for foreground; W, N for background) [Rosenfeld 1966,
 *      cited in Sec. 1], and every background pixel on the image border with
 *      node 0;
 *   2. canonical ids: the exterior is 0, every other component is numbered by
 *      the raster rank of its first pixel;
 *   3. features by direct summation over pixels;
 *   4. the tree by breadth-first search over the region adjacency graph from
 *      the exterior; under the 8/4 connectivity pair that graph is a tree
 *      (the adjacency tree of Rosenfeld 1979, cited in Sec. 1), which the
 *      oracle checks (|edges| = n - 1, all nodes reached);
 *   5. Euler number = #foreground components - #holes, where the holes are
 *      all background components except the exterior.
 *
 * Readings where the paper is silent (stated again in the design notes):
 *   - nonzero pixel = foreground;
 *   - the exterior frame surrounds all four sides (the paper's unification
 *     epilog only attaches the first and last background run of each row,
 *     which misses background touching the bottom edge; the definition of
 *     "surrounded" in Sec. 3.1 fixes the four-sided reading);
 *   - Sx sums the column index x, Sy sums the row index y;
 *   - an empty exterior has S = Sx = Sy = 0 and bbox
 *     (INT32_MAX, -1, INT32_MAX, -1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ECAPACITY (-3)
#define ORC_ENOTTREE (-4)

/* feature record layout of the oracle (its own, independent of the library):
 * 7 int64 per component: xmin, xmax, ymin, ymax, S, Sx, Sy */
#define ORC_NF 7

static int64_t find_root(int64_t *par, int64_t a) {
  while (par[a] != a) {
    par[a] = par[par[a]]; /* path halving */
    a = par[a];
  }
  return a;
}

static void unite(int64_t *par, int64_t a, int64_t b) {
  a = find_root(par, a);
  b = find_root(par, b);
  if (a == b) return;
  if (a < b) par[b] = a;
  else par[a] = b;
}

/* open-addressing set of undirected edges (a < b), packed into a uint64 */
typedef struct {
  uint64_t *slot;
  int64_t cap; /* power of two */
  int64_t n;
} edge_set;

static uint64_t mix64(uint64_t z) {
  z ^= z >> 33;
  z *= 0xff51afd7ed558ccdULL;
  z ^= z >> 33;
  z *= 0xc4ceb9fe1a85ec53ULL;
  z ^= z >> 33;
  return z;
}

static int edge_set_grow(edge_set *s);

/* returns 1 if inserted, 0 if present, -1 on allocation failure */
static int edge_set_add(edge_set *s, int64_t a, int64_t b) {
  uint64_t key = ((uint64_t)a << 32) | (uint64_t)b; /* a, b < 2^31 */
  if ((s->n + 1) * 2 > s->cap)
    if (edge_set_grow(s)) return -1;
  uint64_t m = (uint64_t)s->cap - 1;
  uint64_t i = mix64(key) & m;
  for (;;) {
    if (s->slot[i] == UINT64_MAX) {
      s->slot[i] = key;
      s->n++;
      return 1;
    }
    if (s->slot[i] == key) return 0;
    i = (i + 1) & m;
  }
}

static int edge_set_grow(edge_set *s) {
  int64_t ncap = s->cap ? s->cap * 2 : 1024;
  uint64_t *ns = (uint64_t *)malloc((size_t)ncap * sizeof(uint64_t));
  if (!ns) return -1;
  memset(ns, 0xff, (size_t)ncap * sizeof(uint64_t));
  uint64_t m = (uint64_t)ncap - 1;
  for (int64_t k = 0; k < s->cap; k++) {
    uint64_t key = s->slot[k];
    if (key == UINT64_MAX) continue;
    uint64_t i = mix64(key) & m;
    while (ns[i] != UINT64_MAX) i = (i + 1) & m;
    ns[i] = key;
  }
  free(s->slot);
  s->slot = ns;
  s->cap = ncap;
  return 0;
}

/*
 * oracle_label: label `img` (h rows of w bytes, row stride `pitch` bytes).
 * Outputs (all host memory, caller-allocated):
 *   labels [h*w]       canonical id per pixel, row-major, dense (stride w)
 *   feat   [cap*7]     per id: xmin, xmax, ymin, ymax, S, Sx, Sy
 *   parent [cap]       inclusion tree; parent[0] = -1
 *   color  [cap]       1 = foreground, 0 = background; color[0] = 0
 *   euler  [1]         Euler number
 * Returns n_labels (>= 1) on success, or a negative ORC_* code.  When
 * n_labels > cap, returns ORC_ECAPACITY and leaves the tables unspecified.
 * Any of feat / parent / color may be NULL to skip that table (the tree is
 * still built and checked).
 */
int64_t oracle_label_conn(const uint8_t *img, int32_t w, int32_t h, int64_t pitch,
                          int32_t *labels, int64_t cap, int64_t *feat,
                          int32_t *parent, uint8_t *color, int64_t *euler,
                          int32_t fg8);

int64_t oracle_label(const uint8_t *img, int32_t w, int32_t h, int64_t pitch,
                     int32_t *labels, int64_t cap, int64_t *feat,
                     int32_t *parent, uint8_t *color, int64_t *euler) {
  return oracle_label_conn(img, w, h, pitch, labels, cap, feat, parent, color, euler, 1);
}

/*
 * oracle_label_conn: the same with the connectivity pair chosen: fg8 = 1 is
 * 8-adjacent foreground / 4-adjacent background (the default above); fg8 = 0
 * the complementary pair, 4-adjacent foreground / 8-adjacent background
 * (the note on the connectivity pair after the unification algorithm,
 * Sec. 3.2).  Everything else is unchanged: the frame is background, the
 * region adjacency graph is built from 4-adjacent pairs (a diagonal contact
 * between the two colours always comes with a 4-adjacent one), and under
 * either pair that graph is a tree.
 */
int64_t oracle_label_conn(const uint8_t *img, int32_t w, int32_t h, int64_t pitch,
                          int32_t *labels, int64_t cap, int64_t *feat,
                          int32_t *parent, uint8_t *color, int64_t *euler,
                          int32_t fg8) {
  if (!img || !labels || !euler || w <= 0 || h <= 0 || pitch < w) return ORC_EINVAL;
  int64_t n = (int64_t)w * h;
  if (n >= INT32_MAX) return ORC_EINVAL;

  int64_t *par = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  if (!par) return ORC_ENOMEM;
  for (int64_t i = 0; i <= n; i++) par[i] = i;

#define FG(yy, xx) (img[(int64_t)(yy) * pitch + (xx)] != 0)
#define NODE(yy, xx) (1 + (int64_t)(yy) * w + (xx))

  /* 1. raster union pass (both polarities) */
  for (int32_t y = 0; y < h; y++) {
    for (int32_t x = 0; x < w; x++) {
      int64_t me = NODE(y, x);
      int v = FG(y, x);
      int diag = fg8 ? v : !v; /* this colour is 8-adjacent */
      /* W and N for both colours; NW and NE for the 8-adjacent colour */
      if (x > 0 && FG(y, x - 1) == v) unite(par, me, NODE(y, x - 1));
      if (y > 0) {
        if (FG(y - 1, x) == v) unite(par, me, NODE(y - 1, x));
        if (diag && x > 0 && FG(y - 1, x - 1) == v) unite(par, me, NODE(y - 1, x - 1));
        if (diag && x + 1 < w && FG(y - 1, x + 1) == v) unite(par, me, NODE(y - 1, x + 1));
      }
      if (!v && (x == 0 || y == 0 || x == w - 1 || y == h - 1)) unite(par, me, 0);
    }
  }

  /* 2. canonical ids: exterior 0, then raster rank of first pixel.
   * Reuse `par`: after this pass par[root] holds -(id+1) for every root. */
  int64_t next = 1;
  int64_t r0 = find_root(par, 0); /* always 0: union by minimum index */
  par[r0] = -1;                   /* id 0 */
  for (int64_t p = 0; p < n; p++) {
    int64_t a = p + 1;
    while (par[a] >= 0 && par[a] != a) a = par[a];
    int64_t id;
    if (par[a] < 0) {
      id = -par[a] - 1;
    } else { /* a is a root seen for the first time */
      id = next++;
      par[a] = -(id + 1);
    }
    if (a != p + 1) par[p + 1] = a; /* later pixels reach the root in one step */
    labels[p] = (int32_t)id;
  }
  free(par);
  int64_t nl = next;

  if (nl > cap || nl - 1 > INT32_MAX) {
    return ORC_ECAPACITY;
  }

  /* 3. colour and features by direct summation */
  int64_t *F = feat;
  int64_t *Fown = NULL;
  if (!F) {
    Fown = (int64_t *)malloc((size_t)nl * ORC_NF * sizeof(int64_t));
    if (!Fown) return ORC_ENOMEM;
    F = Fown;
  }
  uint8_t *C = color;
  uint8_t *Cown = NULL;
  if (!C) {
    Cown = (uint8_t *)malloc((size_t)nl);
    if (!Cown) { free(Fown); return ORC_ENOMEM; }
    C = Cown;
  }
  for (int64_t k = 0; k < nl; k++) {
    F[k * ORC_NF + 0] = INT32_MAX;
    F[k * ORC_NF + 1] = -1;
    F[k * ORC_NF + 2] = INT32_MAX;
    F[k * ORC_NF + 3] = -1;
    F[k * ORC_NF + 4] = 0;
    F[k * ORC_NF + 5] = 0;
    F[k * ORC_NF + 6] = 0;
    C[k] = 0;
  }
  for (int32_t y = 0; y < h; y++) {
    for (int32_t x = 0; x < w; x++) {
      int64_t k = labels[(int64_t)y * w + x];
      int64_t *f = F + k * ORC_NF;
      if (x < f[0]) f[0] = x;
      if (x > f[1]) f[1] = x;
      if (y < f[2]) f[2] = y;
      if (y > f[3]) f[3] = y;
      f[4] += 1;
      f[5] += x;
      f[6] += y;
      if (k != 0) C[k] = FG(y, x) ? 1 : 0;
    }
  }

  /* 4. tree: region adjacency graph over 4-adjacent pixel pairs with
   * different ids, plus the exterior frame for foreground border pixels;
   * breadth-first search from the exterior. */
  int rc = 0;
  edge_set es = {0, 0, 0};
  int64_t *deg = NULL, *off = NULL, *adj = NULL, *queue = NULL, *par_out = NULL;
  for (int32_t y = 0; y < h && rc == 0; y++) {
    for (int32_t x = 0; x < w; x++) {
      int64_t k = labels[(int64_t)y * w + x];
      if (x + 1 < w) {
        int64_t q = labels[(int64_t)y * w + x + 1];
        if (q != k && edge_set_add(&es, k < q ? k : q, k < q ? q : k) < 0) { rc = ORC_ENOMEM; break; }
      }
      if (y + 1 < h) {
        int64_t q = labels[(int64_t)(y + 1) * w + x];
        if (q != k && edge_set_add(&es, k < q ? k : q, k < q ? q : k) < 0) { rc = ORC_ENOMEM; break; }
      }
      if (k != 0 && (x == 0 || y == 0 || x == w - 1 || y == h - 1)) {
        /* only foreground can touch the frame without being the exterior */
        if (edge_set_add(&es, 0, k) < 0) { rc = ORC_ENOMEM; break; }
      }
    }
  }
  if (rc == 0 && es.n != nl - 1) rc = ORC_ENOTTREE;
  if (rc == 0) {
    deg = (int64_t *)calloc((size_t)nl, sizeof(int64_t));
    off = (int64_t *)malloc((size_t)(nl + 1) * sizeof(int64_t));
    adj = (int64_t *)malloc((size_t)(2 * es.n + 1) * sizeof(int64_t));
    queue = (int64_t *)malloc((size_t)nl * sizeof(int64_t));
    par_out = (int64_t *)malloc((size_t)nl * sizeof(int64_t));
    if (!deg || !off || !adj || !queue || !par_out) rc = ORC_ENOMEM;
  }
  if (rc == 0) {
    for (int64_t s = 0; s < es.cap; s++) {
      uint64_t key = es.slot[s];
      if (key == UINT64_MAX) continue;
      deg[key >> 32]++;
      deg[key & 0xffffffffULL]++;
    }
    off[0] = 0;
    for (int64_t k = 0; k < nl; k++) off[k + 1] = off[k] + deg[k];
    for (int64_t k = 0; k < nl; k++) deg[k] = off[k];
    for (int64_t s = 0; s < es.cap; s++) {
      uint64_t key = es.slot[s];
      if (key == UINT64_MAX) continue;
      int64_t a = (int64_t)(key >> 32), b = (int64_t)(key & 0xffffffffULL);
      adj[deg[a]++] = b;
      adj[deg[b]++] = a;
    }
    for (int64_t k = 0; k < nl; k++) par_out[k] = -2; /* unvisited */
    par_out[0] = -1;
    int64_t qh = 0, qt = 0;
    queue[qt++] = 0;
    while (qh < qt) {
      int64_t u = queue[qh++];
      for (int64_t e = off[u]; e < off[u + 1]; e++) {
        int64_t v = adj[e];
        if (par_out[v] == -2) {
          par_out[v] = u;
          queue[qt++] = v;
        }
      }
    }
    if (qt != nl) rc = ORC_ENOTTREE;
    if (rc == 0 && parent)
      for (int64_t k = 0; k < nl; k++) parent[k] = (int32_t)par_out[k];
  }

  /* 5. Euler number */
  if (rc == 0) {
    int64_t nfg = 0, nbg = 0;
    for (int64_t k = 0; k < nl; k++) {
      if (C[k]) nfg++;
      else nbg++;
    }
    *euler = nfg - (nbg - 1);
  }

  free(es.slot);
  free(deg);
  free(off);
  free(adj);
  free(queue);
  free(par_out);
  free(Fown);
  free(Cown);
#undef FG
#undef NODE
  return rc == 0 ? nl : rc;
}
