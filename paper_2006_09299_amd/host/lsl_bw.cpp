// lsl_bw.cpp -- single-thread host implementation of LSL-BW (liblslbw.so).
//
// The paper's own CPU algorithm (Lemaitre & Lacassagne 2020), kept as a
// like-for-like CPU comparison for the GPU path: segment detection
// (Sec. 2, Algorithm 1), B&W unification with initial adjacency (Sec. 3.2,
// Algorithm 2), forward transitive closure with the adjacency tree and
// optional hole filling (Algorithm 3), relabeling (Algorithm 4).  Interface
// and readings: include/lslbw.h.  Shares no code with the GPU library or
// with the test oracle.
#include "../../include/lslbw.h"

#include <stdlib.h>
#include <string.h>
#include <time.h>
#include <x86intrin.h>

#include <new>

namespace {

struct Feat {  // same layout as lslbw_feature_t
  int32_t xmin, xmax, ymin, ymax;
  int64_t S, Sx, Sy;
};
static_assert(sizeof(Feat) == sizeof(lslbw_feature_t), "feature layout");

inline void feat_empty(Feat& f) {
  f.xmin = 0x7FFFFFFF;
  f.xmax = -1;
  f.ymin = 0x7FFFFFFF;
  f.ymax = -1;
  f.S = f.Sx = f.Sy = 0;
}
// ComputeFeatures(i, j0, j1) of the run [j0, j1) on row i
inline void feat_run(Feat& f, int i, int j0, int j1) {
  const int64_t n = j1 - j0;
  f.xmin = j0;
  f.xmax = j1 - 1;
  f.ymin = f.ymax = i;
  f.S = n;
  f.Sx = (int64_t)(j0 + j1 - 1) * n / 2;
  f.Sy = (int64_t)i * n;
}
// F <- F u f
inline void feat_merge(Feat& F, const Feat& f) {
  if (f.xmin < F.xmin) F.xmin = f.xmin;
  if (f.xmax > F.xmax) F.xmax = f.xmax;
  if (f.ymin < F.ymin) F.ymin = f.ymin;
  if (f.ymax > F.ymax) F.ymax = f.ymax;
  F.S += f.S;
  F.Sx += f.Sx;
  F.Sy += f.Sy;
}

}  // namespace

struct lslbw_ctx {
  int32_t w, h;
  // provisional labels: equivalence table T, initial adjacency I, colour,
  // features F, final (canonical) id C
  int64_t lcap;
  int32_t* T;
  int32_t* I;
  uint8_t* col;
  Feat* F;
  int32_t* C;
  // runs of every row (kept for the relabeling): boundaries RLC and the
  // absolute label ERA of every run, row i at offset off[i]
  int32_t* RLC;
  int32_t* ERA;
  int64_t* off;
  int32_t* ner;
  // per-pixel relative labels of the current and the previous row, and the
  // virtual background row above row 0
  int32_t* ER[2];
  int32_t* ER0;
};

namespace {

inline int32_t find(const int32_t* T, int32_t e) {
  while (T[e] != e) e = T[e];
  return e;
}

bool grow(lslbw_ctx* c) {
  const int64_t n = c->lcap * 2;
  void* t = realloc(c->T, sizeof(int32_t) * n);
  if (!t) return false;
  c->T = (int32_t*)t;
  t = realloc(c->I, sizeof(int32_t) * n);
  if (!t) return false;
  c->I = (int32_t*)t;
  t = realloc(c->col, n);
  if (!t) return false;
  c->col = (uint8_t*)t;
  t = realloc(c->F, sizeof(Feat) * n);
  if (!t) return false;
  c->F = (Feat*)t;
  t = realloc(c->C, sizeof(int32_t) * n);
  if (!t) return false;
  c->C = (int32_t*)t;
  c->lcap = n;
  return true;
}

// Algorithm 1: runs of row X; RLC[0..ner], ER[0..w-1]; returns ner.
inline int segments(const uint8_t* X, int w, int32_t* RLC, int32_t* ER) {
  RLC[0] = 0;
  int er = 0;
  int x1 = 0;
  for (int j = 0; j < w; j++) {
    const int x0 = X[j] != 0;
    RLC[er + 1] = j;
    er += x0 ^ x1;
    ER[j] = er;
    x1 = x0;
  }
  RLC[er + 1] = w;
  return er + 1;
}

// Algorithm 2 for row i against the row above; returns false when the
// label tables could not grow.
template <bool FEAT, bool FG8>
inline bool unify(lslbw_ctx* c, int i, const int32_t* ERp, const int32_t* ERAp, int32_t& ne) {
  const int w = c->w;
  const int32_t* RLCi = c->RLC + c->off[i];
  int32_t* ERAi = c->ERA + c->off[i];
  const int n = c->ner[i];
  int ers = 0;
  if (RLCi[1] == 0) {  // run 0 (background) is empty: the row starts with foreground
    ERAi[0] = 0;
    ers = 1;
  }
  for (int er = ers; er < n; er++) {
    int j0 = RLCi[er], j1 = RLCi[er + 1];
    const int p = er & 1;            // 1: foreground run
    const int c8 = FG8 ? p : p ^ 1;  // this run's colour is 8-adjacent
    Feat f;
    if (FEAT) feat_run(f, i, j0, j1);
    j0 = j0 - c8 > 0 ? j0 - c8 : 0;
    j1 = j1 + c8 < w ? j1 + c8 : w;
    int er0 = ERp[j0];
    int er1 = ERp[j1 - 1];
    er0 += (er0 & 1) ^ p;  // first / last run above of the same colour
    er1 -= (er1 & 1) ^ p;
    if (er1 >= er0) {
      int32_t a = find(c->T, ERAp[er0]);
      for (int k = er0 + 2; k <= er1; k += 2) {
        const int32_t ak = find(c->T, ERAp[k]);
        if (a < ak) c->T[ak] = a;
        if (a > ak) {
          c->T[a] = ak;
          a = ak;
        }
      }
      ERAi[er] = a;
      if (FEAT) feat_merge(c->F[a], f);
    } else {  // new label; its initial adjacency is the run on its left
      if (ne == c->lcap && !grow(c)) return false;
      ERAi[er] = ne;
      c->T[ne] = ne;
      c->I[ne] = er > 0 ? ERAi[er - 1] : 0;
      c->col[ne] = (uint8_t)p;
      if (FEAT) c->F[ne] = f;
      ne++;
    }
  }
  // the first and the last background runs touch the frame: exterior
  int32_t a = find(c->T, ERAi[0]);
  c->T[a] = 0;
  if (n & 1) {
    a = find(c->T, ERAi[n - 1]);
    c->T[a] = 0;
  }
  if (i == c->h - 1) {  // the frame's bottom side: every background run of the last row
    for (int er = 2; er < n; er += 2) {
      a = find(c->T, ERAi[er]);
      c->T[a] = 0;
    }
  }
  return true;
}

// Algorithm 3 (label 0, the exterior, is left alone: its parent is -1)
template <bool FEAT, bool FILL>
inline void closure(lslbw_ctx* c, int32_t ne) {
  int32_t* T = c->T;
  int32_t* I = c->I;
  for (int32_t e = 1; e < ne; e++) {
    int32_t a = T[e];
    if (FILL && a == e) {
      const int32_t s = I[e];  // surrounding component
      if (T[s] > 0) a = T[e] = s;
    }
    if (a < e) {
      const int32_t r = T[a];
      T[e] = r;
      if (FEAT) feat_merge(c->F[r], c->F[e]);
    } else {
      I[e] = T[I[e]];
    }
  }
}

template <bool FEAT, bool FG8>
bool scan_rows(lslbw_ctx* c, const uint8_t* img, int64_t pitch, int32_t& ne) {
  static const int32_t era_virtual[1] = {0};
  for (int i = 0; i < c->h; i++) {
    int32_t* ERi = c->ER[i & 1];
    const int n = segments(img + (int64_t)i * pitch, c->w, c->RLC + c->off[i], ERi);
    c->ner[i] = n;
    c->off[i + 1] = c->off[i] + n + 1;
    const int32_t* ERp = i ? c->ER[(i - 1) & 1] : c->ER0;
    const int32_t* ERAp = i ? c->ERA + c->off[i - 1] : era_virtual;
    if (!unify<FEAT, FG8>(c, i, ERp, ERAp, ne)) return false;
  }
  return true;
}

}  // namespace

extern "C" int lslbw_create(int32_t w, int32_t h, lslbw_ctx_t** out) {
  if (!out || w < 1 || h < 1 || (int64_t)w * h >= 0x7FFFFFFFll) return LSLBW_EINVAL;
  lslbw_ctx* c = new (std::nothrow) lslbw_ctx;
  if (!c) return LSLBW_ENOMEM;
  memset(c, 0, sizeof(*c));
  c->w = w;
  c->h = h;
  c->lcap = (int64_t)w * h / 4 + w + 2;
  const int64_t runs = (int64_t)h * (w + 2);
  c->T = (int32_t*)malloc(sizeof(int32_t) * c->lcap);
  c->I = (int32_t*)malloc(sizeof(int32_t) * c->lcap);
  c->col = (uint8_t*)malloc(c->lcap);
  c->F = (Feat*)malloc(sizeof(Feat) * c->lcap);
  c->C = (int32_t*)malloc(sizeof(int32_t) * c->lcap);
  c->RLC = (int32_t*)malloc(sizeof(int32_t) * runs);
  c->ERA = (int32_t*)malloc(sizeof(int32_t) * runs);
  c->off = (int64_t*)malloc(sizeof(int64_t) * (h + 1));
  c->ner = (int32_t*)malloc(sizeof(int32_t) * h);
  c->ER[0] = (int32_t*)malloc(sizeof(int32_t) * w);
  c->ER[1] = (int32_t*)malloc(sizeof(int32_t) * w);
  c->ER0 = (int32_t*)calloc(w, sizeof(int32_t));
  if (!c->T || !c->I || !c->col || !c->F || !c->C || !c->RLC || !c->ERA || !c->off || !c->ner || !c->ER[0] ||
      !c->ER[1] || !c->ER0) {
    lslbw_destroy(c);
    return LSLBW_ENOMEM;
  }
  *out = c;
  return LSLBW_OK;
}

extern "C" void lslbw_destroy(lslbw_ctx_t* c) {
  if (!c) return;
  free(c->T);
  free(c->I);
  free(c->col);
  free(c->F);
  free(c->C);
  free(c->RLC);
  free(c->ERA);
  free(c->off);
  free(c->ner);
  free(c->ER[0]);
  free(c->ER[1]);
  free(c->ER0);
  delete c;
}

extern "C" int lslbw_label(lslbw_ctx_t* c, const uint8_t* img, int64_t pitch, int32_t flags, int32_t* labels,
                           lslbw_feature_t* feat, int32_t* parent, uint8_t* color, int64_t cap, int64_t* counts,
                           lslbw_time_t* t) {
  if (!c || !img || !counts || pitch < c->w || cap < 0 || (flags & ~31)) return LSLBW_EINVAL;
  timespec ts0, ts1;
  clock_gettime(CLOCK_MONOTONIC, &ts0);
  const uint64_t tsc0 = __rdtsc();

  const bool FEAT = (flags & LSLBW_FEATURES) != 0, FILL = (flags & LSLBW_FILL) != 0;
  const bool FG8 = (flags & LSLBW_FG4) == 0;
  // label 0: the exterior
  c->T[0] = 0;
  c->I[0] = -1;
  c->col[0] = 0;
  feat_empty(c->F[0]);
  c->off[0] = 0;
  int32_t ne = 1;

  // step 1: segment detection and unification, row by row
  bool ok;
  if (FEAT) ok = FG8 ? scan_rows<true, true>(c, img, pitch, ne) : scan_rows<true, false>(c, img, pitch, ne);
  else ok = FG8 ? scan_rows<false, true>(c, img, pitch, ne) : scan_rows<false, false>(c, img, pitch, ne);
  if (!ok) return LSLBW_ENOMEM;

  // step 2: transitive closure (adjacency tree, optional hole filling)
  if (FEAT) FILL ? closure<true, true>(c, ne) : closure<true, false>(c, ne);
  else FILL ? closure<false, true>(c, ne) : closure<false, false>(c, ne);

  // final ids: roots compacted in increasing order; tables of the roots
  int32_t* C = c->C;
  C[0] = 0;
  if (cap > 0) {
    if (parent) parent[0] = -1;
    if (color) color[0] = 0;
    if (FEAT && feat) memcpy(&feat[0], &c->F[0], sizeof(Feat));
  }
  int32_t nl = 1;
  int64_t nfg = 0, nbg = 0;
  for (int32_t e = 1; e < ne; e++) {
    const int32_t r = c->T[e];
    if (r != e) {
      C[e] = C[r];
      continue;
    }
    const int32_t id = nl++;
    C[e] = id;
    if (c->col[e]) nfg++;
    else nbg++;
    if (id < cap) {
      if (parent) parent[id] = C[c->I[e]];
      if (color) color[id] = c->col[e];
      if (FEAT && feat) memcpy(&feat[id], &c->F[e], sizeof(Feat));
    }
  }
  counts[0] = nl;
  counts[1] = (flags & LSLBW_EULER) ? nfg - nbg : 0;

  // step 3: relabeling, run by run
  if ((flags & LSLBW_RELABEL) && labels) {
    const int w = c->w;
    for (int i = 0; i < c->h; i++) {
      const int32_t* RLCi = c->RLC + c->off[i];
      const int32_t* ERAi = c->ERA + c->off[i];
      int32_t* E = labels + (int64_t)i * w;
      const int n = c->ner[i];
      int j0 = RLCi[0];
      for (int er = 0; er < n; er++) {
        const int32_t r = C[ERAi[er]];
        const int j1 = RLCi[er + 1];
        for (int j = j0; j < j1; j++) E[j] = r;
        j0 = j1;
      }
    }
  }

  const uint64_t tsc1 = __rdtsc();
  clock_gettime(CLOCK_MONOTONIC, &ts1);
  if (t) {
    t->tsc = tsc1 - tsc0;
    t->ns = (uint64_t)((ts1.tv_sec - ts0.tv_sec) * 1000000000ll + (ts1.tv_nsec - ts0.tv_nsec));
  }
  return LSLBW_OK;
}
