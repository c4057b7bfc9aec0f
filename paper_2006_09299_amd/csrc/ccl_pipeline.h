// ccl_pipeline.h -- HIP kernels and launch sequence of the black-and-white
// run-based connected-component labeling + analysis path for gfx950.
//
// Method: Lemaitre & Lacassagne, "A new run-based Connected Component
// Labeling for efficiently analyzing and processing holes" (2020).
//   * runs (segments) of alternating background / foreground per row
//     (Sec. 2, segment detection);
//   * foreground 8-adjacent, background 4-adjacent unification of runs of
//     consecutive rows by union of equivalence classes with the minimum as
//     representative (Sec. 3.2, B&W unification: widening by one pixel for
//     foreground, parity fix, min-propagation / min-extraction);
//   * features bounding box, S, Sx, Sy accumulated per run and merged into
//     the representative (Sec. 1; ComputeFeatures and the feature merge of
//     the transitive closure);
//   * inclusion tree by initial adjacency: the surrounding of a component is
//     the component of the pixel just left of its first pixel in raster order
//     (Sec. 3.1; pointed at the final root by the closure);
//   * Euler number = #foreground components - #holes (Sec. 1, Table 1);
//   * relabeling of every pixel with its final label (Sec. 3.2, relabeling).
//
// GPU decomposition (no sequential row scan): the image is cut into TH x TW
// tiles, one workgroup per tile.
//   k_tile_export : pack the tile to bits, extract runs, unite runs of
//                   consecutive rows in LDS, find which local components touch
//                   the tile border, export them as "border nodes" with their
//                   partial features, count interior components per row, and
//                   leave the tile state (bits, root masks, the root ordinal of
//                   every run) for k_tile_emit.  A one-colour tile skips the
//                   union-find: one border node, features in closed form.
//   k_seam_local  : unite the seams inside each SUP x SUP group of tiles
//                   (super-tile) with a 16-bit union-find in LDS over the
//                   group's border nodes; every non-root node is pointed at
//                   its super-tile root.
//   k_border_merge: unite border nodes across the remaining tile edges
//                   (seams between super-tiles: horizontal and vertical,
//                   foreground diagonals across corners) and background on
//                   the image border with the exterior node; lock-free
//                   union-find in HBM (link by compare-and-swap).
//   k_reduce_roots: point every border node at its root; the root takes the
//                   minimum raster key and the sum of the partial features
//                   (LDS hash per group of tiles first; k_reduce_direct is the
//                   variant with direct atomics).
//   k_leaders     : which border node holds its component's first pixel; rank
//                   of that pixel among the components starting in the same
//                   row of the same tile.
//   k_scan_*      : exclusive scan of component starts over (row, tile column)
//                   in raster order -> canonical id base of every such cell
//                   (block totals; then every block adds the totals of the
//                   image's earlier blocks and scans its own cells).
//   k_border_canon: canonical id of every border node; features of the
//                   components crossing tiles.
//   k_tile_emit   : from the tile state: canonical id of every run, the label
//                   image, features / colour / parent of every component the
//                   tile owns and its Euler number contribution.
//
// Canonical ids: the exterior (background connected to the image border,
// through a one-pixel background frame on all four sides) is 0; every other
// component is numbered by the raster rank of its first pixel.
//
// The kernels use only HIP device features; the launch sequence is written
// against a small launcher interface so that the same source drives the HIP
// runtime (ccl.hip).
#pragma once

#include <stdint.h>
#include <type_traits>

namespace ccl {

typedef unsigned long long u64;
typedef uint32_t u32;
typedef uint16_t u16;
typedef uint8_t u8;

// Output record, bit-identical to ccl_feature_t of include/ccl.h.
struct Feature {
  int32_t xmin, xmax, ymin, ymax;
  int64_t S, Sx, Sy;
};

// One image of a launch.  All pointers are device memory.
struct ImgDesc {
  const u8* img;
  int64_t pitch;
  int32_t w, h;
  int32_t* labels;   // [h*w] or null
  Feature* feat;     // [cap] or null
  int32_t* parent;   // [cap] or null
  u8* color;         // [cap] or null
  int64_t cap;
  int64_t* counts;   // [2]: n_labels, Euler number
  int32_t ntx, nty;  // tiles across / down
  int32_t flags;     // bit0: 16-byte input loads, bit1: 16-byte label stores
  int32_t nblk;      // scan blocks of this image
  int64_t tile0;     // first global tile index
  int64_t node0;     // global id of this image's exterior node
  int64_t c0;        // offset of the (row, tile column) count grid
  int64_t blk0;      // first scan block
  int64_t it0;       // first border-merge work item
  int64_t nit;       // border-merge work items
  int64_t s0;        // first super-tile (SUP x SUP tiles) of this image
  uint32_t check;    // batches: digest of the variant and the batch totals the
                     // descriptor was placed for (kernels of another launch
                     // shape leave it alone)
  uint32_t pad_;
};

enum { DF_VEC_IN = 1, DF_VEC_LAB = 2 };

// Four labels with one 16-byte store that does not keep the line in the
// caches: the label image is written once and never read back by the path.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
__device__ inline void store_labels4(int32_t* dst, int32_t a, int32_t b, int32_t c, int32_t e) {
  i32x4 v = {a, b, c, e};
  __builtin_nontemporal_store(v, reinterpret_cast<i32x4*>(dst));
}

// Workspace views (device memory), shared by all images of a launch.
struct Work {
  int32_t* gpar;     // [nodes] union-find parent of border nodes
  int32_t* gkey;     // [nodes] raster index of the node's first pixel
  int32_t* gminkey;  // [nodes] at roots: minimum key of the class
  int32_t* grank;    // [nodes] bits 0-15 rank / interior-before, 16-21 row, 31 leader
  int32_t* rcanon;   // [nodes] at roots: rank of the component among those starting in its first pixel's cell
  int32_t* ncanon;   // [nodes] canonical id of the node's component (before K5: the cell of its first pixel)
  Feature* gacc;     // [nodes] partial features; at roots the class sum
  int32_t* nbt;      // [tiles] border nodes per tile
  // border arrays, the two sides of a tile next to each other (indexed by
  // side rather than by pointer: a per-lane choice of pointer makes the
  // compiler load it from the kernel arguments through vector memory)
  u16* bidx_h;       // [tiles][2][TW] border node index of every top (0) / bottom (1) row pixel
  u16* bidx_v;       // [tiles][2][TH] left (0) / right (1) column
  u64* bits_h;       // [tiles][2][WPR] foreground bits of the top / bottom row
  u64* bits_lr;      // [tiles*2] left column (bit = row), right column
  int32_t* cgrid;    // [sum h*ntx] per (row, tile column): starts, then base ids
  int32_t* bsum;     // [scan blocks]
  // tile state handed from K1 to K6, tile raster order inside each tile
  int32_t* tinfo;    // [tiles] general tile: runs << 2; one-colour tile: 1 + colour
  u64* tstate;       // [tiles*3*NW] foreground bits, root masks, border-root masks
  u16* tord;         // [tiles*N] root ordinal of every run, by run rank
                     // (border roots first, then interior roots, raster order)
  int32_t* rcol;     // [tiles*TH] canonical id of the component at each row's last pixel
  uint32_t k1_stride;  // K1's tile order: block b labels tile (b * k1_stride) mod tiles
  int32_t rh_group;    // tiles per k_reduce_roots workgroup (a power of two)
};

// Tile of this workgroup: block b takes tile (b * stride) mod tiles, a
// permutation when the stride is coprime to the tile count (1: raster order).
__device__ inline int64_t tile_of_block(uint32_t stride) {
  if (stride == 1u) return blockIdx.x;
  return (int64_t)(((uint64_t)blockIdx.x * stride) % gridDim.x);
}

constexpr u32 HI = 0x80000000u;
// Each image's node block starts with its exterior node followed by EXT_REP
// accumulators of the exterior's features: the root reduction spreads the
// exterior's partial sums over them by workgroup (one address taking the
// atomics of every workgroup serialises them), and k_border_canon adds them up.
constexpr int EXT_REP = 32;
constexpr int SCAN_T = 256;             // threads of the scan kernels (whole waves)
static_assert(SCAN_T % 64 == 0, "the block scan works in whole waves");
constexpr int SCAN_B = SCAN_T * 4;      // entries per scan block

// Merge schedule: SUP_ tiles per side of a super-tile (its inner seams are
// merged in LDS by k_seam_local, the rest by k_border_merge); RHT_ tiles per
// workgroup of the root reduction (0: chosen per launch, at most 128 for
// tiles of more than 4096 pixels, else 32).
template <int TH_, int TW_, int NT_ = 256, bool FG8_ = true, int SUP_ = 4, int RHT_ = 0>
struct Tile {
  static constexpr int TH = TH_;
  static constexpr int TW = TW_;
  static constexpr int WPR = TW / 64;      // 64-bit words per row
  static constexpr int NW = TH * WPR;      // words per tile
  static constexpr int N = TH * TW;        // pixel positions per tile
  static constexpr int CPR = TW / 16;      // 16-pixel chunks per row
  static constexpr int NCH = TH * CPR;     // chunks per tile
  static constexpr int BCAP = 2 * (TH + TW);  // >= border pixels >= border nodes
  static constexpr int NT = NT_;           // threads per tile workgroup
  // connectivity pair: 8-adjacent foreground / 4-adjacent background, or
  // the complementary pair (the unification's widening moves to background)
  static constexpr bool FG8 = FG8_;
  static constexpr int CAPI = N >= 8192 ? 512 : 256;  // interior accumulators per pass
  static constexpr int SUP = SUP_;
  static constexpr int RHT = RHT_ ? RHT_ : (N > 4096 ? 128 : 32);
  static constexpr bool RHT_AUTO = RHT_ == 0;
  static_assert(SUP >= 2 && SUP <= 8, "super-tile side");
  static_assert(RHT >= 1 && RHT <= 256, "root-reduction group");
  static_assert(TW % 64 == 0 && TW <= 256, "tile width (a row rank fits 8 bits)");
  static_assert(TH >= 1 && TH <= 64, "tile height (a column of the tile fits one wave)");
  static_assert(NT >= 128 && NT % 64 == 0, "at least two waves per tile");
  static_assert(N < 65536, "positions must fit 16 bits");
  static_assert((long long)N * (TW - 1) < (1ll << 24), "packed Sx field");
  static_assert((long long)N * (TH - 1) < (1ll << 24), "packed Sy field");
  static_assert(NW <= 256, "prefix scan width");
};

// ---------------------------------------------------------------------------
// small device helpers

__device__ inline int clz64(u64 v) { return __builtin_clzll(v); }
__device__ inline int ctz32(u32 v) { return __builtin_ctz(v); }
__device__ inline int popc64(u64 v) { return __builtin_popcountll(v); }
__device__ inline u64 low_mask(int b) { return b >= 64 ? ~0ull : ((1ull << b) - 1ull); }  // bits < b
__device__ inline u64 valid_mask(int j, int width) {  // bits x of word j with 64*j + x < width
  int n = width - 64 * j;
  return n >= 64 ? ~0ull : (n <= 0 ? 0ull : ((1ull << n) - 1ull));
}
// nonzero bytes of a dword -> 4 bits (byte k -> bit k)
__device__ inline u32 nz4(u32 d) {
  u32 t = (((d & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | d) & 0x80808080u;
  return ((t >> 7) * 0x10204080u) >> 28;
}

// LDS written by some lanes of a wave is read by others after this point
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  (void)__ballot(1);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// sum over the 64 lanes of a wave (every lane gets it)
__device__ inline int wave_sum(int v) {
  const int lane = (int)(threadIdx.x & 63u);
  for (int dl = 32; dl >= 1; dl >>= 1) v += __shfl(v, lane ^ dl, 64);
  return v;
}

__device__ inline u32 ld_wg(const u32* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void st_wg(u32* p, u32 v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void st_ag(int32_t* p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
// A load that is issued where it is written: relaxed atomic loads are not
// moved to their first use the way plain loads are.
template <class V>
__device__ inline V ld_now(const V* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Union-find in LDS over tile positions, 16-bit entries: union by minimum,
// path halving.  A root is linked with compare-and-swap (on the 32-bit word
// holding its entry) only while it is still a root, so a tree never loses
// members; path halving only ever writes an ancestor into a non-root.
// Concurrent finds and links are therefore safe.
__device__ inline u32 ld16(const u16* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ inline void st16(u16* p, u32 v) { __hip_atomic_store(p, (u16)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }

// Where entry i lives: the identity, or (tile union-find over positions)
// bits 1-3 of the position XORed with bits 7-9, so that the lanes of a wave,
// which hold consecutive 16-pixel chunks of several rows and touch the same
// offset in each, reach different LDS banks.  Bit 0 is kept: the two entries
// of a 32-bit word stay together (linking swaps one of them by CAS).
struct IdMap {
  __device__ u32 operator()(u32 i) const { return i; }
};
struct SwzMap {
  __device__ u32 operator()(u32 i) const { return i ^ (((i >> 7) & 7u) << 1); }
};
__device__ inline u32 swz(u32 p) { return SwzMap()(p); }

// link root b under a; false if b is no longer a root
template <class M = IdMap>
__device__ inline bool llink(u16* par, u32 a, u32 b, M m = M()) {
  u32* w = reinterpret_cast<u32*>(par + (m(b) & ~1u));
  const int sh = (int)(b & 1u) * 16;
  u32 old = ld_wg(w);
  for (;;) {
    if (((old >> sh) & 0xFFFFu) != b) return false;
    u32 nw = (old & ~(0xFFFFu << sh)) | (a << sh);
    u32 prev = atomicCAS(w, old, nw);
    if (prev == old) return true;
    old = prev;  // the word changed (possibly only the other entry): look again
  }
}
// unite the classes of a and b: both walks advance together, two levels
// per step with path halving; the loads are unconditional (a walk that has
// reached its root reads it again) so that the four of a step overlap
template <class M = IdMap>
__device__ inline void lunion(u16* par, u32 a, u32 b, M m = M()) {
  for (;;) {
    for (;;) {
      u32 pa = ld16(par + m(a)), pb = ld16(par + m(b));
      u32 ga = ld16(par + m(pa)), gb = ld16(par + m(pb));
      if (ga != pa) st16(par + m(a), ga);  // a is not a root: halve
      if (gb != pb) st16(par + m(b), gb);
      const bool fa = ga == pa, fb = gb == pb;  // pa / pb is a root
      a = ga;
      b = gb;
      if (a == b) return;
      if (fa && fb) break;
    }
    if (a > b) {
      u32 t = a;
      a = b;
      b = t;
    }
    if (llink(par, a, b, m)) return;  // else b was linked meanwhile: retry
  }
}
// read-only walk to the root (no writes)
template <class M = IdMap>
__device__ inline u32 lroot(const u16* par, u32 x, M m = M()) {
  u32 p = ld16(par + m(x));
  while (p != x) {
    x = p;
    p = ld16(par + m(x));
  }
  return x;
}

// Union-find in HBM over border nodes (same scheme; links and compression
// writes at agent scope, reads through the caches).
// Find with path compression.  Every entry points to a smaller index unless
// it is a root, so both walks strictly decrease and end.  The second walk
// points the entries above the root found at that root.
// Concurrency with unions (gunion): roots are linked by compare-and-swap only
// while they are roots, so trees only grow and the root found stays an
// ancestor of every entry of the walked path.  The walk writes only into
// entries it has just read as non-roots (a non-root never becomes a root
// again, so no write can meet a link), only ever writes r < x, and stops at
// the first index <= r.  Without concurrent unions all writes of a class
// carry its final root.
// A read may return an older value of an entry: that is an older ancestor
// (entries only ever move up their tree), so walks stay correct; a node seen
// as a root that has been linked meanwhile makes the link fail, and the
// failed compare-and-swap returns the entry's current value, from which the
// walk goes on (each failure climbs at least one level, so unions end).
__device__ inline int ld_wk(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline int gfind(int32_t* gp, int x) {
  int r = x;
  int p = ld_wk(&gp[r]);
  while (p != r) {
    r = p;
    p = ld_wk(&gp[r]);
  }
  while (x > r) {
    int n = ld_wk(&gp[x]);
    if (n <= r || n == x) break;
    st_ag(&gp[x], r);
    x = n;
  }
  return r;
}
__device__ inline void gunion(int32_t* gp, int a, int b) {
  for (;;) {
    a = gfind(gp, a);
    b = gfind(gp, b);
    if (a == b) return;
    if (a > b) { int t = a; a = b; b = t; }
    // link the larger root under the smaller one, only if it is still a root;
    // on failure b holds the entry's current value (a strict ancestor)
    if (__hip_atomic_compare_exchange_strong(&gp[b], &b, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

// Pixel pairs of two consecutive rows that unite runs (B&W unification).
// m0: lower row bits, m1: upper row bits, *p / *n: the words before / after,
// V: valid bits of the word (pixels inside the row), pfull: the word before
// is entirely inside the row.  Returns:
//   vert: one bit per maximal interval of same-colour vertical pairs (both
//         colours: 4-adjacency), unite run(lower, x) with run(upper, x);
//   da:   foreground diagonal to the upper right, unite with run(upper, x+1)
//         (the lower run ends at x, the upper run starts at x+1);
//   db:   foreground diagonal to the upper left, unite with run(upper, x-1).
// Vn: valid bits of the word after.  With the complementary connectivity
// pair (FG8 false) the diagonals are those of the background: the same
// formulas on the background bits of the valid pixels.
struct PairMasks { u64 vert, da, db; };
template <bool FG8>
__device__ inline PairMasks pair_masks(u64 m0, u64 m1, u64 m0p, u64 m1p, u64 m0n, u64 m1n, u64 V, bool pfull,
                                       u64 Vn) {
  PairMasks r;
  u64 F = m0 & m1, Fp = m0p & m1p;
  u64 Fv = F & ~((F << 1) | (Fp >> 63));
  u64 B = ~m0 & ~m1 & V;
  u64 Bp = pfull ? (~m0p & ~m1p) : 0ull;
  u64 Bv = B & ~((B << 1) | (Bp >> 63));
  r.vert = Fv | Bv;
  if (!FG8) {  // diagonal colour: background
    m0 = ~m0 & V;
    m1 = ~m1 & V;
    m0n = ~m0n & Vn;
    m1n = ~m1n & Vn;
    m0p = pfull ? ~m0p : 0ull;
    m1p = pfull ? ~m1p : 0ull;
  }
  u64 R1 = (m1 >> 1) | (m1n << 63), R0 = (m0 >> 1) | (m0n << 63);
  u64 L1 = (m1 << 1) | (m1p >> 63), L0 = (m0 << 1) | (m0p >> 63);
  r.da = m0 & ~m1 & R1 & ~R0 & V;
  r.db = m0 & ~m1 & L1 & ~L0 & V;
  return r;
}

// Diagonal contacts across a vertical seam between rows y-1 and y: a, b the
// pixels left / right of the seam in row y, c, dd in row y-1 (1 =
// foreground).  Only the diagonal colour's contacts count, and only where
// the crossing diagonal has the other colour (else a 4-path joins them).
template <bool FG8>
__device__ inline bool diag_right_up(int a, int b, int c, int dd) {  // (right, y) with (left, y-1)
  return FG8 ? (b && c && !a && !dd) : (!b && !c && a && dd);
}
template <bool FG8>
__device__ inline bool diag_left_up(int a, int b, int c, int dd) {  // (left, y) with (right, y-1)
  return FG8 ? (a && dd && !b && !c) : (!a && !dd && b && c);
}

// packed per-component accumulators: S | Sx << 16 | Sy << 40 (tile-local
// coordinates), bounding box extremes; ymin is the row of the first pixel.
// Acc (K1's border partials) keeps each extreme in a word of its own; AccP
// (K6's interior components) both x extremes in one word, so that the
// record takes 16 bytes and K6's LDS leaves room for four workgroups per CU.
struct Acc {
  u64 s;
  u32 xmin, xmax, ymax;
};
struct AccP {
  u64 s;
  u32 xr;  // xmin | xmax << 16
  u32 ymax;
};

__device__ inline u64 seg_pack(int ly, int s, int e) {
  u64 n = (u64)(e - s);
  u64 sx = (u64)(s + e - 1) * n / 2;  // sum of x over [s, e)
  u64 sy = (u64)ly * n;
  return n | (sx << 16) | (sy << 40);
}

// ---------------------------------------------------------------------------
// shared tile labeling (k_tile_export and k_tile_emit run the same phases)

template <class T>
struct TileSmem {
  u64 bits[T::NW];   // foreground bits
  u64 st[T::NW];     // run starts
  u64 bflag[T::NW];  // roots whose component touches the tile border
  u64 rootm[T::NW];  // roots (position p with par[p] == p at a run start)
  // union-find over positions ly * TW + x (only run starts are used); once
  // the roots are known, the root ordinal of every run start
  alignas(16) u16 par[T::N];
  u16 bpre[T::NW];   // border roots before word (tile raster order)
  u16 ipre[T::NW];   // interior roots before word
  u16 spre[T::NW];   // run starts before word
  int nb, nint, nruns;
};

template <class T>
__device__ inline int run_start(const TileSmem<T>& s, int ly, int x) {  // x of the run holding (ly, x)
  const u64* row = &s.st[ly * T::WPR];
  int j = x >> 6;
  u64 m = row[j] & (~0ull >> (63 - (x & 63)));
  if constexpr (T::WPR == 2) {
    // bit 0 of a row's first word is always a start: with two words per
    // row the fallback is that word, taken by selects rather than a branch
    const u64 m0 = row[0];
    const bool fb = m == 0ull;
    m = fb ? m0 : m;
    j = fb ? 0 : j;
  } else if (T::WPR > 2) {
    const u64 mp = row[j > 0 ? j - 1 : 0];  // read ahead: the usual fallback
    if (!m) {
      m = mp;
      j--;
      while (!m) m = row[--j];  // ends: bit 0 of word 0 is always a start
    }
  }
  return (j << 6) + 63 - clz64(m);
}

template <class T>
__device__ inline int bidx_of(const TileSmem<T>& s, int r) {  // r: border root position
  int wd = r >> 6;
  return s.bpre[wd] + popc64(s.bflag[wd] & s.rootm[wd] & low_mask(r & 63));
}
template <class T>
__device__ inline int iord_of(const TileSmem<T>& s, int r) {  // r: interior root position
  int wd = r >> 6;
  return s.ipre[wd] + popc64(~s.bflag[wd] & s.rootm[wd] & low_mask(r & 63));
}

// Geometry of one tile of an image.
struct TileGeom {
  int64_t lt;      // tile index inside its image
  int tx, ty;      // tile column / row
  int x0, y0;      // first pixel
  int tw, th;      // pixels inside the image
};
template <class T>
__device__ inline TileGeom tile_geom(const ImgDesc& d, int64_t gt) {
  TileGeom g;
  g.lt = gt - d.tile0;
  g.tx = (int)(g.lt % d.ntx);
  g.ty = (int)(g.lt / d.ntx);
  g.x0 = g.tx * T::TW;
  g.y0 = g.ty * T::TH;
  g.tw = d.w - g.x0 < T::TW ? d.w - g.x0 : T::TW;
  g.th = d.h - g.y0 < T::TH ? d.h - g.y0 : T::TH;
  return g;
}

// Image bytes of one thread's 16-pixel chunks (and the byte before the chunk
// for a wave's first lane), all requested before any is used.  Chunks that
// are not whole 16-byte aligned vectors are read at use.
template <class T>
struct TileFetch {
  static constexpr int K = (T::NCH + T::NT - 1) / T::NT;
  // a wave's first lane holds a chunk that starts a row unless the chunks of
  // a row do not divide 64 (then it reads the byte before its chunk); the
  // byte loads are issued after all vector loads (each load's use waits for
  // every earlier one)
  static constexpr bool PREV = 64 % T::CPR != 0;
  uint4 v[K];
  u32 prevb[PREV ? K : 1];
};

template <class T>
__device__ inline void tile_fetch(TileFetch<T>& f, const ImgDesc& d, const TileGeom& g) {
  const int tid = threadIdx.x;
  const bool vec_in = (d.flags & DF_VEC_IN) != 0;
#pragma unroll
  for (int k = 0; k < TileFetch<T>::K; k++) {
    const int c = k * T::NT + tid;
    const int ly = c / T::CPR, cx = (c % T::CPR) * 16;
    const bool in = c < T::NCH && ly < g.th && cx < g.tw;
    const u8* src = d.img + (int64_t)(g.y0 + ly) * d.pitch + (g.x0 + cx);
    uint4 v;
    v.x = v.y = v.z = v.w = 0u;
    if (in && vec_in && cx + 16 <= g.tw) v = *reinterpret_cast<const uint4*>(src);
    f.v[k] = v;
  }
  if constexpr (TileFetch<T>::PREV) {
#pragma unroll
    for (int k = 0; k < TileFetch<T>::K; k++) {
      const int c = k * T::NT + tid;
      const int ly = c / T::CPR, cx = (c % T::CPR) * 16;
      const bool in = c < T::NCH && ly < g.th && cx < g.tw;
      const u8* src = d.img + (int64_t)(g.y0 + ly) * d.pitch + (g.x0 + cx);
      f.prevb[k] = in && cx > 0 && (tid & 63) == 0 ? (u32)src[-1] : 0u;
    }
  }
}

// Phase 1: pack + runs.  Returns 1 + colour for a one-colour tile, else 0.
// Ends with a barrier; afterwards bits/st are valid and par[p] == p at every
// run start p (general tile).
template <class T>
__device__ int tile_pack(TileSmem<T>& s, const TileFetch<T>& f, const ImgDesc& d, const TileGeom& g) {
  static_assert(T::NCH % 64 == 0 || T::NCH < 64, "whole waves per chunk loop");
  const int tid = threadIdx.x;
  const int tw = g.tw, th = g.th;
  const bool vec_in = (d.flags & DF_VEC_IN) != 0;
  // 1. bytes -> 16 bits per chunk; run starts (the pixel before the chunk
  // comes from the lane holding the previous chunk, or from memory at a
  // wave's first lane); par[p] = p at every run start; vote on a one-colour
  // tile
  bool all0 = true, all1 = true;
#pragma unroll
  for (int k = 0; k < TileFetch<T>::K; k++) {
    const int c0 = k * T::NT;
    const int c = c0 + tid;
    if (c0 + (tid & ~63) >= T::NCH) break;  // whole waves leave together
    const int ly = c / T::CPR, cc = c % T::CPR, cx = cc * 16;
    const bool in = c < T::NCH && ly < th && cx < tw;
    u32 m = 0;
    if (in) {
      if (vec_in && cx + 16 <= tw) {
        const uint4 v = f.v[k];
        m = nz4(v.x) | (nz4(v.y) << 4) | (nz4(v.z) << 8) | (nz4(v.w) << 12);
      } else {
        const u8* src = d.img + (int64_t)(g.y0 + ly) * d.pitch + (g.x0 + cx);
        int n = tw - cx < 16 ? tw - cx : 16;
        for (int q = 0; q < n; q++) m |= (u32)(src[q] != 0) << q;
      }
    }
    u32 prev = __shfl_up(m, 1, 64);
    if (c >= T::NCH) continue;
    reinterpret_cast<u16*>(s.bits)[c] = (u16)m;
    u32 e = 0;
    if (in) {
      u32 carry;
      if (cc == 0) carry = ~m & 1u;
      else if (TileFetch<T>::PREV && (tid & 63) == 0) carry = f.prevb[TileFetch<T>::PREV ? k : 0] != 0u;
      else carry = prev >> 15;
      const u32 vm = (u32)valid_mask(0, tw - cx) & 0xFFFFu;
      e = (m ^ ((m << 1) | carry)) & vm;
      all0 = all0 && (m & vm) == 0;
      all1 = all1 && (m & vm) == vm;
    }
    // par[p] = p for the chunk's 16 positions (only run starts are ever
    // read): two 16-byte stores instead of a loop over the run starts, whose
    // count varies from lane to lane.  The chunk fills one aligned block of
    // 16 entries, which swz permutes: slot i holds position p0 + (i ^ 2 sw).
    {
      const u32 p0 = (u32)c * 16u;  // = ly * TW + cx
      const u32 sw = (p0 >> 7) & 7u;
      const u32 base = p0 | ((p0 + 1u) << 16);
      uint4 lo, hi;
      lo.x = base + ((0u ^ sw) * 2u) * 0x10001u;
      lo.y = base + ((1u ^ sw) * 2u) * 0x10001u;
      lo.z = base + ((2u ^ sw) * 2u) * 0x10001u;
      lo.w = base + ((3u ^ sw) * 2u) * 0x10001u;
      hi.x = base + ((4u ^ sw) * 2u) * 0x10001u;
      hi.y = base + ((5u ^ sw) * 2u) * 0x10001u;
      hi.z = base + ((6u ^ sw) * 2u) * 0x10001u;
      hi.w = base + ((7u ^ sw) * 2u) * 0x10001u;
      uint4* dst = reinterpret_cast<uint4*>(&s.par[p0]);
      dst[0] = lo;
      dst[1] = hi;
    }
    reinterpret_cast<u16*>(s.st)[c] = (u16)e;
  }
  for (int i = tid; i < T::NW; i += T::NT) s.bflag[i] = 0;
  const int u0 = __syncthreads_and(all0);
  const int u1 = __syncthreads_and(all1);
  return u0 || u1 ? (u1 ? 2 : 1) : 0;
}

// Phases 2-5 of a general tile: unite, flatten, border flags and roots,
// prefix counts.  Ends with a barrier; afterwards par[p] is the root
// position of every run start p, bflag/rootm/bpre/ipre/spre/nb/nint/nruns
// are valid.
template <class T>
__device__ void tile_unite(TileSmem<T>& s, u32* stage_all, int stage_words, int tw, int th) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  // 2. unite runs of rows ly-1, ly (all row pairs at once).  Each lane finds
  // the union points of one 16-pixel chunk; the wave then lists them in LDS
  // (x | row << 10 | kind << 16) and works through the list 64 at a time, so
  // that its iterations follow the wave's total instead of its busiest lane.
  const int scap = stage_words / (T::NT / 64);
  u32* stage = stage_all + (tid >> 6) * scap;
#pragma unroll
  for (int k = 0; k < (T::NCH + T::NT - 1) / T::NT; k++) {
    if (k * T::NT + (tid & ~63) >= T::NCH) break;  // whole waves leave together
    const int c = k * T::NT + tid;
    const int ly = c / T::CPR, cc = c % T::CPR;
    // bits 0-15: vertical; 16-31: diagonal up-right; 32-47: diagonal up-left
    u64 pts = 0;
    int xb = 0;
    if (c < T::NCH && ly > 0 && ly < th && cc * 16 < tw) {
      const int j = cc >> 2, sh = (cc & 3) * 16;
      const u64* B0 = &s.bits[ly * T::WPR];
      const u64* B1 = &s.bits[(ly - 1) * T::WPR];
      u64 m0 = B0[j], m1 = B1[j];
      u64 m0p = j ? B0[j - 1] : 0ull, m1p = j ? B1[j - 1] : 0ull;
      u64 m0n = j + 1 < T::WPR ? B0[j + 1] : 0ull, m1n = j + 1 < T::WPR ? B1[j + 1] : 0ull;
      PairMasks pm = pair_masks<T::FG8>(m0, m1, m0p, m1p, m0n, m1n, valid_mask(j, tw), j > 0, valid_mask(j + 1, tw));
      pts = ((pm.vert >> sh) & 0xFFFFull) | (((pm.da >> sh) & 0xFFFFull) << 16) |
            (((pm.db >> sh) & 0xFFFFull) << 32);
      xb = j * 64 + sh;
    }
    if (!__ballot(popc64(pts) > 2)) {
      // few points per lane in this wave: each lane does its own
      while (pts) {
        const int kk = __builtin_ctzll(pts);
        pts &= pts - 1;
        const int x = xb + (kk & 15);
        const int xu = x + (kk >> 4 == 1) - (kk >> 4 == 2);
        lunion(s.par, (u32)(ly * T::TW + run_start(s, ly, x)), (u32)((ly - 1) * T::TW + run_start(s, ly - 1, xu)),
               SwzMap());
      }
      continue;
    }
    for (;;) {
      // wave prefix of the points still to do
      const int cnt = popc64(pts);
      int inc = cnt;
      for (int dl = 1; dl < 64; dl <<= 1) {
        int t = __shfl_up(inc, dl, 64);
        if (lane >= dl) inc += t;
      }
      const int total = __shfl(inc, 63, 64);
      if (total == 0) break;
      const int n = total < scap ? total : scap;
      int take = n - (inc - cnt);
      take = take < 0 ? 0 : (take > cnt ? cnt : take);
      for (int q = inc - cnt; take > 0; take--, q++) {
        const int kk = __builtin_ctzll(pts);
        pts &= pts - 1;
        stage[q] = (u32)(xb + (kk & 15)) | ((u32)ly << 10) | ((u32)(kk >> 4) << 16);
      }
      wave_sync();
      for (int i = lane; i < n; i += 64) {
        const u32 e = stage[i];
        const int x = (int)(e & 1023u), row = (int)((e >> 10) & 63u), kind = (int)(e >> 16);
        const int xu = x + (kind == 1) - (kind == 2);
        lunion(s.par, (u32)(row * T::TW + run_start(s, row, x)), (u32)((row - 1) * T::TW + run_start(s, row - 1, xu)),
               SwzMap());
      }
      wave_sync();  // the list is rewritten next round
    }
  }
  __syncthreads();

  // 3. flatten: every run start points at its root (own entry written
  // only); root masks; the roots of components touching the tile border
  // (runs of the first and last rows, each row's first run and its last
  // run, which holds the last pixel) are flagged
  for (int c = tid; c < T::NCH; c += T::NT) {
    const int ly = c / T::CPR, cc = c % T::CPR;
    const int j = cc >> 2, sh = (cc & 3) * 16;
    const u64* strow = &s.st[ly * T::WPR];
    u32 m = ly < th ? (u32)(strow[j] >> sh) & 0xFFFFu : 0u;
    // the row's last run starts in this chunk when no start follows it
    bool later = sh < 48 && (strow[j] >> (sh + 16)) != 0ull;
    for (int jj = j + 1; jj < T::WPR; jj++) later = later || strow[jj] != 0ull;
    const u32 last = m && !later ? 1u << (31 - __builtin_clz(m)) : 0u;
    const u32 edge = ly == 0 || ly == th - 1 ? 0xFFFFu : ((cc == 0 ? 1u : 0u) | last);
    u32 rm = 0;
    while (m) {
      const int k = ctz32(m);
      m &= m - 1;
      const u32 p = (u32)(ly * T::TW + j * 64 + sh + k);
      const u32 r = lroot(s.par, p, SwzMap());
      if (r == p) rm |= 1u << k;
      else st16(&s.par[swz(p)], r);
      if ((edge >> k) & 1u) atomicOr(&s.bflag[r >> 6], 1ull << (r & 63));
    }
    reinterpret_cast<u16*>(s.rootm)[c] = (u16)rm;
  }
  __syncthreads();

  // 5. exclusive prefix counts of border roots, interior roots and run
  // starts over words
  if (tid < 64) {
    u32 cb = 0, ci = 0, cs = 0;
    for (int base = 0; base < T::NW; base += 64) {
      int wd = base + tid;
      u64 rm = wd < T::NW ? s.rootm[wd] : 0ull;
      u64 bf = wd < T::NW ? s.bflag[wd] : 0ull;
      u32 nb = (u32)popc64(rm & bf), ni = (u32)popc64(rm & ~bf);
      u32 v = nb | (ni << 16);  // both counts <= 4096 per 64 words
      u32 vs = wd < T::NW ? (u32)popc64(s.st[wd]) : 0u;
      u32 inc = v, incs = vs;
      for (int d = 1; d < 64; d <<= 1) {
        u32 t = __shfl_up(inc, d, 64);
        u32 ts = __shfl_up(incs, d, 64);
        if (tid >= d) {
          inc += t;
          incs += ts;
        }
      }
      u32 exc = inc - v;
      if (wd < T::NW) {
        s.bpre[wd] = (u16)(cb + (exc & 0xFFFFu));
        s.ipre[wd] = (u16)(ci + (exc >> 16));
        s.spre[wd] = (u16)(cs + incs - vs);
      }
      u32 tot = __shfl(inc, 63, 64);
      cb += tot & 0xFFFFu;
      ci += tot >> 16;
      cs += __shfl(incs, 63, 64);
    }
    if (tid == 0) {
      s.nb = (int)cb;
      s.nint = (int)ci;
      s.nruns = (int)cs;
    }
  }
  __syncthreads();
}

// Segments of one 16-pixel chunk: calls f(run_start_x, seg_begin, seg_end).
template <class T, class Fn>
__device__ inline void for_segments(const TileSmem<T>& s, int ly, int cc, int tw, Fn f) {
  int cs = cc * 16;
  if (cs >= tw) return;
  int ce = cs + 16 < tw ? cs + 16 : tw;
  int j = cc >> 2, sh = (cc & 3) * 16;
  u32 m = ((u32)(s.st[ly * T::WPR + j] >> sh) & 0xFFFFu) & ~1u;
  int start = run_start(s, ly, cs);
  int x = cs;
  for (;;) {
    int nx = m ? cs + ctz32(m) : ce;
    f(start, x, nx);
    if (!m) break;
    m &= m - 1;
    start = nx;
    x = nx;
  }
}

__device__ inline void acc_init(Acc& a) {
  a.s = 0;
  a.xmin = 0xFFFFu;
  a.xmax = 0;
  a.ymax = 0;
}
__device__ inline void acc_init(AccP& a) {
  a.s = 0;
  a.xr = 0xFFFFu;  // xmin 0xFFFF, xmax 0
  a.ymax = 0;
}
// Segments of one row summed in registers before they go to a shared
// accumulator: consecutive segments (in x order) of one component.
struct RowSum {
  int o;       // accumulator index, -1: none
  u64 s;       // packed S | Sx | Sy
  u32 xmin, xmax;
};
// the extremes only ever move outwards: an atomic is needed only when the
// value read does not already include this one (reads of one address by
// many lanes are served at once, atomics on it one after another)
__device__ inline void acc_x(Acc& a, u32 xmin, u32 xmax) {
  if (xmin < ld_wg(&a.xmin)) atomicMin(&a.xmin, xmin);
  if (xmax > ld_wg(&a.xmax)) atomicMax(&a.xmax, xmax);
}
__device__ inline void acc_x(AccP& a, u32 xmin, u32 xmax) {
  // both in one word: merged by compare-and-swap, which succeeds or returns
  // a value that already moved one of them outwards
  u32 old = ld_wg(&a.xr);
  while (xmin < (old & 0xFFFFu) || xmax > (old >> 16)) {
    const u32 lo = xmin < (old & 0xFFFFu) ? xmin : (old & 0xFFFFu);
    const u32 hi = xmax > (old >> 16) ? xmax : (old >> 16);
    const u32 prev = atomicCAS(&a.xr, old, lo | (hi << 16));
    if (prev == old) break;
    old = prev;
  }
}
template <class A>
__device__ inline void rowsum_flush(RowSum& r, A* acc, int ly) {
  if (r.o < 0) return;
  A& a = acc[r.o];
  atomicAdd(&a.s, r.s);
  acc_x(a, r.xmin, r.xmax);
  if ((u32)ly > ld_wg(&a.ymax)) atomicMax(&a.ymax, (u32)ly);
  r.o = -1;
}
template <class A>
__device__ inline void rowsum_add(RowSum& r, A* acc, int o, int ly, int s0, int e0) {
  if (o != r.o) {
    rowsum_flush(r, acc, ly);
    r.o = o;
    r.s = 0;
    r.xmin = (u32)s0;
  }
  r.s += seg_pack(ly, s0, e0);
  r.xmax = (u32)(e0 - 1);
}

__device__ inline u32 acc_xmin(const Acc& a) { return a.xmin; }
__device__ inline u32 acc_xmax(const Acc& a) { return a.xmax; }
__device__ inline u32 acc_xmin(const AccP& a) { return a.xr & 0xFFFFu; }
__device__ inline u32 acc_xmax(const AccP& a) { return a.xr >> 16; }
template <class A>
__device__ inline Feature acc_abs(const A& a, int ly_min, int x0, int y0) {
  Feature f;
  int64_t S = (int64_t)(a.s & 0xFFFFull);
  int64_t sx = (int64_t)((a.s >> 16) & 0xFFFFFFull);
  int64_t sy = (int64_t)(a.s >> 40);
  f.xmin = (int32_t)acc_xmin(a) + x0;
  f.xmax = (int32_t)acc_xmax(a) + x0;
  f.ymin = ly_min + y0;
  f.ymax = (int32_t)a.ymax + y0;
  f.S = S;
  f.Sx = sx + S * x0;
  f.Sy = sy + S * y0;
  return f;
}

// ---------------------------------------------------------------------------
// descriptor sources: one image by value, or an array in device memory

struct OneImage {
  ImgDesc d;
  __device__ const ImgDesc& by_tile(int64_t) const { return d; }
  __device__ const ImgDesc& by_item(int64_t) const { return d; }
  __device__ const ImgDesc& by_block(int64_t) const { return d; }
  __device__ const ImgDesc& by_index(int64_t) const { return d; }
  __device__ const ImgDesc& by_super(int64_t) const { return d; }
  __device__ int64_t count() const { return 1; }
  __device__ bool ok(const ImgDesc&) const { return true; }
};

struct ManyImages {
  const ImgDesc* ds;
  int32_t n;
  uint32_t check;  // what every descriptor of this launch must carry
  // last descriptor whose field `first` is <= v (descriptors sorted by it)
  template <class Get>
  __device__ const ImgDesc& search(int64_t v, Get get) const {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (get(ds[mid]) <= v) lo = mid;
      else hi = mid - 1;
    }
    return ds[lo];
  }
  __device__ const ImgDesc& by_tile(int64_t t) const { return search(t, [](const ImgDesc& d) { return d.tile0; }); }
  __device__ const ImgDesc& by_item(int64_t i) const { return search(i, [](const ImgDesc& d) { return d.it0; }); }
  __device__ const ImgDesc& by_block(int64_t b) const { return search(b, [](const ImgDesc& d) { return d.blk0; }); }
  __device__ const ImgDesc& by_index(int64_t i) const { return ds[i]; }
  __device__ const ImgDesc& by_super(int64_t v) const { return search(v, [](const ImgDesc& d) { return d.s0; }); }
  __device__ int64_t count() const { return n; }
  __device__ bool ok(const ImgDesc& d) const { return d.check == check; }
};

template <class T>
__device__ inline int64_t tile_node_base(const ImgDesc& d, int64_t lt) {  // slot 0 of local tile lt
  return d.node0 + 1 + EXT_REP + lt * T::BCAP;
}

// ---------------------------------------------------------------------------
// K1: tile labeling and export of border nodes

// One tile after phase 1 (uni: tile_pack's result).
template <class T>
__device__ void export_tile(TileSmem<T>& s, Acc* bacc, const ImgDesc& d, const TileGeom& g, int64_t gt, int uni,
                            const Work& wk) {
  const int64_t lt = g.lt;
  const int tx = g.tx;
  const int x0 = g.x0, y0 = g.y0, tw = g.tw, th = g.th;
  const int tid = threadIdx.x;

  if (lt == 0 && tid <= EXT_REP) {  // per-image state read by later kernels
    Feature e;
    e.xmin = 0x7FFFFFFF; e.xmax = -1; e.ymin = 0x7FFFFFFF; e.ymax = -1;
    e.S = 0; e.Sx = 0; e.Sy = 0;
    wk.gacc[d.node0 + tid] = e;  // the exterior and its accumulators
    if (tid == 0) {
      wk.gpar[d.node0] = (int32_t)d.node0;
      wk.gminkey[d.node0] = -1;
      wk.gkey[d.node0] = -1;
      if (d.counts) d.counts[1] = 0;
    }
  }

  const int64_t nbase = tile_node_base<T>(d, lt);

  if (uni) {
    // one-colour tile: a single border node whose first pixel is (x0, y0),
    // features in closed form, every border pixel maps to node slot 0
    const int col = uni - 1;
    if (tid == 0) {
      int32_t key = (int32_t)((int64_t)y0 * d.w + x0);
      wk.gpar[nbase] = (int32_t)nbase;
      wk.gkey[nbase] = key;
      wk.gminkey[nbase] = key;
      wk.grank[nbase] = 0;
      Feature f;
      f.xmin = x0; f.xmax = x0 + tw - 1; f.ymin = y0; f.ymax = y0 + th - 1;
      f.S = (int64_t)tw * th;
      f.Sx = (int64_t)th * ((int64_t)x0 * tw + (int64_t)tw * (tw - 1) / 2);
      f.Sy = (int64_t)tw * ((int64_t)y0 * th + (int64_t)th * (th - 1) / 2);
      wk.gacc[nbase] = f;
      wk.nbt[gt] = 1;
      wk.tinfo[gt] = uni;
    }
    for (int ly = tid; ly < th; ly += T::NT) wk.cgrid[d.c0 + (int64_t)(y0 + ly) * d.ntx + tx] = 0;
    for (int t = tid; t < 2 * T::TW + 2 * T::TH; t += T::NT) {
      if (t < 2 * T::TW) {
        int x = t % T::TW;
        wk.bidx_h[gt * 2 * T::TW + t] = x < tw ? (u16)0 : (u16)0xFFFFu;
      } else {
        int k = t - 2 * T::TW;
        int ly = k % T::TH;
        wk.bidx_v[gt * 2 * T::TH + k] = ly < th ? (u16)0 : (u16)0xFFFFu;
      }
    }
    for (int t = tid; t < 2 * T::WPR + 2; t += T::NT) {
      if (t < 2 * T::WPR) {
        int j = t % T::WPR;
        wk.bits_h[gt * 2 * T::WPR + t] = col ? valid_mask(j, tw) : 0ull;
      } else {
        wk.bits_lr[gt * 2 + (t - 2 * T::WPR)] = col ? low_mask(th) : 0ull;
      }
    }
    return;
  }

  tile_unite<T>(s, reinterpret_cast<u32*>(bacc), (int)(sizeof(Acc) * T::BCAP / 4), tw, th);

  // 6. root ordinal of every run start (border roots first, then interior
  // roots) into par and into the tile state for K6; border node records;
  // interior roots per row
  const int nb = s.nb;
  u16* to = wk.tord + gt * T::N;
  for (int c = tid; c < T::NCH; c += T::NT) {
    int ly = c / T::CPR, cc = c % T::CPR;
    if (ly >= th) continue;
    int j = cc >> 2, sh = (cc & 3) * 16;
    int wd = ly * T::WPR + j;
    u64 stw = s.st[wd];
    int rank = s.spre[wd] + popc64(stw & low_mask(sh));
    for (u32 m = (u32)(stw >> sh) & 0xFFFFu; m; m &= m - 1) {
      int p = ly * T::TW + j * 64 + sh + ctz32(m);
      u32 r = s.par[swz(p)];
      int o = ((s.bflag[r >> 6] >> (r & 63)) & 1ull) ? bidx_of<T>(s, (int)r) : nb + iord_of<T>(s, (int)r);
      s.par[swz(p)] = (u16)o;  // only this thread reads this entry from here on
      to[rank++] = (u16)o;
    }
    const u64 bmw = s.rootm[wd] & s.bflag[wd];
    const u64 imw = s.rootm[wd] & ~s.bflag[wd];
    const int ib_row = s.ipre[wd] - s.ipre[ly * T::WPR];
    for (u32 m = (u32)(bmw >> sh) & 0xFFFFu; m; m &= m - 1) {
      int k = sh + ctz32(m);
      int x = j * 64 + k;
      int bi = s.bpre[wd] + popc64(bmw & low_mask(k));
      int64_t node = nbase + bi;
      int32_t key = (int32_t)((int64_t)(y0 + ly) * d.w + x0 + x);
      wk.gpar[node] = (int32_t)node;
      wk.gkey[node] = key;
      wk.gminkey[node] = key;
      wk.grank[node] = (ib_row + popc64(imw & low_mask(k))) | (ly << 16);
      acc_init(bacc[bi]);
    }
  }
  for (int ly = tid; ly < th; ly += T::NT) {
    int next = ly + 1 < T::TH ? s.ipre[(ly + 1) * T::WPR] : s.nint;
    wk.cgrid[d.c0 + (int64_t)(y0 + ly) * d.ntx + tx] = next - s.ipre[ly * T::WPR];
  }
  u64* ts = wk.tstate + gt * 3 * T::NW;
  for (int i = tid; i < 3 * T::NW; i += T::NT) {
    int k = i / T::NW, wd = i % T::NW;
    ts[i] = k == 0 ? s.bits[wd] : (k == 1 ? s.rootm[wd] : (s.rootm[wd] & s.bflag[wd]));
  }
  if (tid == 0) {
    wk.nbt[gt] = nb;
    wk.tinfo[gt] = s.nruns << 2;
  }
  __syncthreads();

  // 7. partial features of border components
  for (int c = tid; c < T::NCH; c += T::NT) {
    int ly = c / T::CPR, cc = c % T::CPR;
    if (ly >= th) continue;
    RowSum rs;
    rs.o = -1;
    for_segments<T>(s, ly, cc, tw, [&](int start, int a, int b) {
      int o = s.par[swz(ly * T::TW + start)];
      if (o < nb) rowsum_add(rs, bacc, o, ly, a, b);
    });
    rowsum_flush(rs, bacc, ly);
  }
  __syncthreads();

  // 8. write partial features and the border arrays
  for (int c = tid; c < T::NCH; c += T::NT) {
    int ly = c / T::CPR, cc = c % T::CPR;
    int j = cc >> 2, sh = (cc & 3) * 16;
    int wd = ly * T::WPR + j;
    const u64 bmw = s.rootm[wd] & s.bflag[wd];
    for (u32 m = (u32)(bmw >> sh) & 0xFFFFu; m; m &= m - 1) {
      int bi = s.bpre[wd] + popc64(bmw & low_mask(sh + ctz32(m)));
      wk.gacc[nbase + bi] = acc_abs(bacc[bi], ly, x0, y0);
    }
  }
  for (int t = tid; t < 2 * T::TW + 2 * T::TH; t += T::NT) {
    if (t < 2 * T::TW) {
      int bottom = t >= T::TW;
      int x = t % T::TW;
      int ly = bottom ? th - 1 : 0;
      u16 v = 0xFFFFu;
      if (x < tw) v = s.par[swz(ly * T::TW + run_start(s, ly, x))];
      wk.bidx_h[gt * 2 * T::TW + t] = v;
    } else {
      int k = t - 2 * T::TW;
      int right = k >= T::TH;
      int ly = k % T::TH;
      u16 v = 0xFFFFu;
      if (ly < th) v = s.par[swz(ly * T::TW + (right ? run_start(s, ly, tw - 1) : 0))];
      wk.bidx_v[gt * 2 * T::TH + k] = v;
    }
  }
  for (int t = tid; t < 2 * T::WPR; t += T::NT) {
    wk.bits_h[gt * 2 * T::WPR + t] = t < T::WPR ? s.bits[t] : s.bits[(th - 1) * T::WPR + (t - T::WPR)];
  }
  // left / right column bits (bit = row): one lane per row of waves 0 / 1
  if (tid < 128) {
    const int right = tid >> 6, ly = tid & 63;
    const int x = right ? tw - 1 : 0;
    const bool fg = ly < th && ((s.bits[ly * T::WPR + (x >> 6)] >> (x & 63)) & 1ull);
    const u64 col = __ballot(fg);
    if (ly == 0) wk.bits_lr[gt * 2 + right] = col;
  }
}

template <class T, class Src>
__global__ void __launch_bounds__(T::NT) k_tile_export(Src src, Work wk) {
  __shared__ TileSmem<T> s;
  __shared__ Acc bacc[T::BCAP];
  const int64_t gt = tile_of_block(wk.k1_stride);
  const ImgDesc& d = src.by_tile(gt);
  if (!src.ok(d)) {  // placed for another variant or batch: flag the image
    if (threadIdx.x == 0 && d.counts) d.counts[0] = -1;
    return;
  }
  const TileGeom g = tile_geom<T>(d, gt);
  TileFetch<T> f;
  tile_fetch<T>(f, d, g);
  const int uni = tile_pack<T>(s, f, d, g);
  export_tile<T>(s, bacc, d, g, gt, uni, wk);
}

// ---------------------------------------------------------------------------
// K2: unions across tile seams and with the exterior

template <class T>
__device__ inline u64 seam_bits(const Work& wk, const ImgDesc& d, int tile_row, int jw, bool bottom) {
  int nwr = (d.w + 63) >> 6;
  if (jw < 0 || jw >= nwr) return 0ull;
  int tcol = jw / T::WPR, j = jw % T::WPR;
  int64_t gt = d.tile0 + (int64_t)tile_row * d.ntx + tcol;
  return wk.bits_h[(gt * 2 + (bottom ? 1 : 0)) * T::WPR + j];
}
template <class T>
__device__ inline int seam_node(const Work& wk, const ImgDesc& d, int tile_row, int x, bool bottom) {
  int tcol = x / T::TW;
  int64_t lt = (int64_t)tile_row * d.ntx + tcol;
  int64_t gt = d.tile0 + lt;
  u16 b = wk.bidx_h[(gt * 2 + (bottom ? 1 : 0)) * T::TW + (x % T::TW)];
  return (int)(tile_node_base<T>(d, lt) + b);
}
template <class T>
__device__ inline int col_node(const Work& wk, const ImgDesc& d, int tcol, int y, bool right) {
  int64_t lt = (int64_t)(y / T::TH) * d.ntx + tcol;
  int64_t gt = d.tile0 + lt;
  u16 b = wk.bidx_v[(gt * 2 + (right ? 1 : 0)) * T::TH + (y % T::TH)];
  return (int)(tile_node_base<T>(d, lt) + b);
}
template <class T>
__device__ inline int col_bit(const Work& wk, const ImgDesc& d, int tcol, int y, bool right) {
  int64_t gt = d.tile0 + (int64_t)(y / T::TH) * d.ntx + tcol;
  return (int)((wk.bits_lr[gt * 2 + (right ? 1 : 0)] >> (y % T::TH)) & 1ull);
}

template <class T>
__host__ __device__ inline int64_t merge_items(int w, int h, int ntx, int nty) {
  // horizontal seams on super-tile row edges (every 4 pixels of every
  // word), horizontal seams inside super-tiles (the two edge words of
  // each super-tile column), vertical seams on super-tile column edges
  // (every row), exterior (top / bottom rows by quarter words, left / right
  // columns by row)
  const int64_t nwr = (w + 63) / 64, nstx = (ntx + T::SUP - 1) / T::SUP;
  const int64_t hb = (nty - 1) / T::SUP, hi = (nty - 1) - hb, vb = (ntx - 1) / T::SUP;
  return hb * nwr * 16 + hi * 2 * nstx + vb * h + 8 * nwr + 2 * (int64_t)h;
}

// ---------------------------------------------------------------------------
// K2a: seams inside a super-tile (SUP x SUP tiles) merged in LDS.  The border
// nodes of the super-tile's tiles get local indices (tile k = row * SUP +
// column inside the super-tile, times BCAP, plus the slot), which are in the
// same order as their global ids, so union by minimum agrees with the global
// union-find.  Every union point of a seam between two tiles of the
// super-tile whose two pixels lie in it is done here; k_border_merge does the
// rest (seams on super-tile edges, diagonals leaving a super-tile, the
// exterior).  Afterwards every node points at its local root.

template <class T>
__device__ inline int lnode_of(const Work& wk, const ImgDesc& d, int tx0, int ty0, int tx, int ty, u16 slot) {
  (void)wk;
  (void)d;
  return ((ty - ty0) * T::SUP + (tx - tx0)) * T::BCAP + slot;
}

// threads per super-tile: its items are chains of dependent loads, so more
// of them in flight at once; super-tiles of 8 x 8 tiles (48 KB of LDS for
// 64 x 128 tiles, two workgroups per CU) take 1024
template <class T>
constexpr int sl_threads() { return T::SUP >= 8 ? 1024 : 512; }

template <class T, class Src>
__global__ void __launch_bounds__(sl_threads<T>()) k_seam_local(Src src, Work wk) {
  constexpr int SL_T = sl_threads<T>();
  constexpr int NL = T::SUP * T::SUP * T::BCAP;
  static_assert(NL < 65536 && NL % 2 == 0, "local node index fits 16 bits");
  __shared__ u32 lpw[NL / 2];  // 16-bit entries; 32-bit words for the links
  u16* lp = reinterpret_cast<u16*>(lpw);
  const int tid = threadIdx.x;
  const int64_t gs = blockIdx.x;
  const ImgDesc& d = src.by_super(gs);
  if (!src.ok(d)) return;
  const int64_t ls = gs - d.s0;
  const int nstx = (d.ntx + T::SUP - 1) / T::SUP;
  const int tx0 = (int)(ls % nstx) * T::SUP, ty0 = (int)(ls / nstx) * T::SUP;
  const int ntxs = d.ntx - tx0 < T::SUP ? d.ntx - tx0 : T::SUP;
  const int ntys = d.nty - ty0 < T::SUP ? d.nty - ty0 : T::SUP;
  for (int l = tid; l < NL; l += SL_T) lp[l] = (u16)l;
  __syncthreads();

  const int xs0 = tx0 * T::TW;
  const int xs1 = (tx0 + ntxs) * T::TW < d.w ? (tx0 + ntxs) * T::TW : d.w;  // pixel range [xs0, xs1)
  // horizontal seams between tile rows ty0 + e - 1 and ty0 + e, 16 pixels per item
  const int nchk = (xs1 - xs0 + 15) / 16;
  const int nh = (ntys - 1) * nchk;
  // vertical seams between tile columns tx0 + e - 1 and tx0 + e, one image row per item
  const int y0s = ty0 * T::TH;
  const int rows = (ty0 + ntys) * T::TH < d.h ? (ty0 + ntys) * T::TH - y0s : d.h - y0s;
  const int nv = (ntxs - 1) * rows;
  for (int it = tid; it < nh + nv; it += SL_T) {
    if (it < nh) {
      const int e = ty0 + 1 + it / nchk;
      const int x16 = xs0 + (it % nchk) * 16;
      const int jw = x16 >> 6, sh = x16 & 63;
      u64 m0 = seam_bits<T>(wk, d, e, jw, false), m1 = seam_bits<T>(wk, d, e - 1, jw, true);
      u64 m0p = seam_bits<T>(wk, d, e, jw - 1, false), m1p = seam_bits<T>(wk, d, e - 1, jw - 1, true);
      u64 m0n = seam_bits<T>(wk, d, e, jw + 1, false), m1n = seam_bits<T>(wk, d, e - 1, jw + 1, true);
      PairMasks pm = pair_masks<T::FG8>(m0, m1, m0p, m1p, m0n, m1n, valid_mask(jw, d.w), jw > 0,
                                         valid_mask(jw + 1, d.w));
      u64 pts = ((pm.vert >> sh) & 0xFFFFull) | (((pm.da >> sh) & 0xFFFFull) << 16) |
                (((pm.db >> sh) & 0xFFFFull) << 32);
      while (pts) {
        const int k = __builtin_ctzll(pts);
        pts &= pts - 1;
        const int x = x16 + (k & 15);
        const int xu = x + (k >> 4 == 1) - (k >> 4 == 2);
        if (xu < xs0 || xu >= xs1) continue;  // leaves the super-tile: k_border_merge
        const int64_t gl = d.tile0 + (int64_t)e * d.ntx + x / T::TW;
        const int64_t gu = d.tile0 + (int64_t)(e - 1) * d.ntx + xu / T::TW;
        const int a = lnode_of<T>(wk, d, tx0, ty0, x / T::TW, e, wk.bidx_h[gl * 2 * T::TW + x % T::TW]);
        const int b = lnode_of<T>(wk, d, tx0, ty0, xu / T::TW, e - 1, wk.bidx_h[(gu * 2 + 1) * T::TW + xu % T::TW]);
        lunion(lp, (u32)a, (u32)b);
      }
    } else {
      const int q = it - nh;
      const int e = tx0 + 1 + q / rows, y = y0s + q % rows;
      const int ly = y % T::TH, ty = y / T::TH;
      const int a = col_bit<T>(wk, d, e - 1, y, true), b = col_bit<T>(wk, d, e, y, false);
      int c = -1, dd = -1;
      if (ly > 0) {
        c = col_bit<T>(wk, d, e - 1, y - 1, true);
        dd = col_bit<T>(wk, d, e, y - 1, false);
      }
      const int64_t gL = d.tile0 + (int64_t)ty * d.ntx + (e - 1), gR = d.tile0 + (int64_t)ty * d.ntx + e;
      auto left = [&](int yy) { return lnode_of<T>(wk, d, tx0, ty0, e - 1, ty, wk.bidx_v[(gL * 2 + 1) * T::TH + yy % T::TH]); };
      auto right = [&](int yy) { return lnode_of<T>(wk, d, tx0, ty0, e, ty, wk.bidx_v[gR * 2 * T::TH + yy % T::TH]); };
      if (a == b && !(ly > 0 && c == a && dd == b)) lunion(lp, (u32)left(y), (u32)right(y));
      if (ly > 0) {
        if (diag_right_up<T::FG8>(a, b, c, dd)) lunion(lp, (u32)right(y), (u32)left(y - 1));
        if (diag_left_up<T::FG8>(a, b, c, dd)) lunion(lp, (u32)left(y), (u32)right(y - 1));
      }
    }
  }
  __syncthreads();

  // every node of the super-tile points at its local root
  for (int l = tid; l < NL; l += SL_T) {
    const int k = l / T::BCAP, slot = l % T::BCAP;
    const int tx = tx0 + k % T::SUP, ty = ty0 + k / T::SUP;
    if (tx - tx0 >= ntxs || ty - ty0 >= ntys) continue;
    const int64_t lt = (int64_t)ty * d.ntx + tx;
    if (slot >= wk.nbt[d.tile0 + lt]) continue;
    const u32 r = lroot(lp, (u32)l);
    if (r == (u32)l) continue;
    const int kr = (int)r / T::BCAP, sr = (int)r % T::BCAP;
    const int64_t ltr = (int64_t)(ty0 + kr / T::SUP) * d.ntx + tx0 + kr % T::SUP;
    wk.gpar[tile_node_base<T>(d, lt) + slot] = (int32_t)(tile_node_base<T>(d, ltr) + sr);
  }
}

template <class T, class Src>
__global__ void __launch_bounds__(256) k_border_merge(Src src, Work wk, int64_t total) {
  const int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= total) return;
  const ImgDesc& d = src.by_item(gi);
  if (!src.ok(d)) return;
  int64_t i = gi - d.it0;
  const int nwr = (d.w + 63) >> 6;
  const int ext = (int)d.node0;
  constexpr int SW = T::SUP * T::WPR;  // words per super-tile column
  const int nstx = (d.ntx + T::SUP - 1) / T::SUP;
  const int64_t hb = (d.nty - 1) / T::SUP, hi = (d.nty - 1) - hb, vb = (d.ntx - 1) / T::SUP;
  const int64_t nH = hb * nwr * 16 + hi * 2 * nstx;
  const int64_t nV = vb * d.h;
  if (i < nH) {  // horizontal seam: bottom row of tile row e-1 above top row of tile row e
    int e, jw;
    bool inner;
    u64 part = ~0ull;  // the word's bits this item unites
    if (i < hb * nwr * 16) {  // on a super-tile row edge: 4 pixels of a word
                              // per item (a dense row has up to 32 union
                              // points per word, each a chain of finds: a
                              // quarter word per item was 15 % slower on
                              // random images, a whole word twice as slow)
      const int64_t iw = i >> 4;
      e = T::SUP * (int)(iw / nwr + 1);
      jw = (int)(iw % nwr);
      part = 0xFull << (4 * (int)(i & 15));
      inner = false;
    } else {  // inside super-tiles, merged by k_seam_local except for the
              // diagonals that leave a super-tile column at its edge words
      const int64_t q = (i - hb * nwr * 16) / (2 * nstx);
      const int r = (int)((i - hb * nwr * 16) % (2 * nstx));
      e = (int)(q + 1 + q / (T::SUP - 1));  // the q-th seam index that is not a multiple of T::SUP
      jw = (r >> 1) * SW + ((r & 1) ? SW - 1 : 0);
      if (jw >= nwr) return;
      inner = true;
    }
    u64 m0 = seam_bits<T>(wk, d, e, jw, false), m1 = seam_bits<T>(wk, d, e - 1, jw, true);
    u64 m0p = seam_bits<T>(wk, d, e, jw - 1, false), m1p = seam_bits<T>(wk, d, e - 1, jw - 1, true);
    u64 m0n = seam_bits<T>(wk, d, e, jw + 1, false), m1n = seam_bits<T>(wk, d, e - 1, jw + 1, true);
    PairMasks pm = pair_masks<T::FG8>(m0, m1, m0p, m1p, m0n, m1n, valid_mask(jw, d.w), jw > 0,
                                         valid_mask(jw + 1, d.w));
    int xb = jw * 64;
    u64 m = pm.vert & part;
    pm.da &= part;
    pm.db &= part;
    if (inner) {  // only the diagonals that cross a super-tile column edge
      m = 0;
      pm.da &= (jw % SW == SW - 1) ? (1ull << 63) : 0ull;
      pm.db &= (jw % SW == 0) ? 1ull : 0ull;
    }
    while (m) {
      int x = xb + __builtin_ctzll(m);
      m &= m - 1;
      gunion(wk.gpar, seam_node<T>(wk, d, e, x, false), seam_node<T>(wk, d, e - 1, x, true));
    }
    m = pm.da;
    while (m) {
      int x = xb + __builtin_ctzll(m);
      m &= m - 1;
      gunion(wk.gpar, seam_node<T>(wk, d, e, x, false), seam_node<T>(wk, d, e - 1, x + 1, true));
    }
    m = pm.db;
    while (m) {
      int x = xb + __builtin_ctzll(m);
      m &= m - 1;
      gunion(wk.gpar, seam_node<T>(wk, d, e, x, false), seam_node<T>(wk, d, e - 1, x - 1, true));
    }
    return;
  }
  i -= nH;
  if (i < nV) {  // vertical seam on a super-tile column edge, between tile columns e-1 and e, image row y
    int e = T::SUP * (int)(i / d.h + 1), y = (int)(i % d.h);
    int ly = y % T::TH;
    int a = col_bit<T>(wk, d, e - 1, y, true), b = col_bit<T>(wk, d, e, y, false);
    int c = -1, dd = -1;
    if (ly > 0) {
      c = col_bit<T>(wk, d, e - 1, y - 1, true);
      dd = col_bit<T>(wk, d, e, y - 1, false);
    }
    if (a == b && !(ly > 0 && c == a && dd == b))
      gunion(wk.gpar, col_node<T>(wk, d, e - 1, y, true), col_node<T>(wk, d, e, y, false));
    if (ly > 0) {
      if (diag_right_up<T::FG8>(a, b, c, dd))
        gunion(wk.gpar, col_node<T>(wk, d, e, y, false), col_node<T>(wk, d, e - 1, y - 1, true));
      if (diag_left_up<T::FG8>(a, b, c, dd))
        gunion(wk.gpar, col_node<T>(wk, d, e - 1, y, true), col_node<T>(wk, d, e, y - 1, false));
    }
    return;
  }
  i -= nV;
  if (i < 8 * (int64_t)nwr) {  // image top / bottom row: background runs join the exterior
                                // (one 16-pixel quarter of a word per item)
    const int part = (int)(i & 3);
    i >>= 2;
    bool bottom = i >= nwr;
    int jw = (int)(i % nwr);
    int row = bottom ? d.nty - 1 : 0;
    u64 V = valid_mask(jw, d.w);
    u64 bg = ~seam_bits<T>(wk, d, row, jw, bottom) & V;
    u64 bgp = jw > 0 ? ~seam_bits<T>(wk, d, row, jw - 1, bottom) : 0ull;
    u64 starts = bg & ~((bg << 1) | (bgp >> 63));
    if (jw % T::WPR == 0) starts |= bg & 1ull;  // each tile holds its own piece
    starts &= 0xFFFFull << (16 * part);
    while (starts) {
      int x = jw * 64 + __builtin_ctzll(starts);
      starts &= starts - 1;
      gunion(wk.gpar, seam_node<T>(wk, d, row, x, bottom), ext);
    }
    return;
  }
  i -= 8 * (int64_t)nwr;
  if (i < 2 * (int64_t)d.h) {  // image left / right column
    bool right = i >= d.h;
    int y = (int)(i % d.h);
    int tcol = right ? d.ntx - 1 : 0;
    if (col_bit<T>(wk, d, tcol, y, right)) return;
    if (y % T::TH > 0 && !col_bit<T>(wk, d, tcol, y - 1, right)) return;  // same piece as the row above
    gunion(wk.gpar, col_node<T>(wk, d, tcol, y, right), ext);
  }
}

// ---------------------------------------------------------------------------
// K3: final roots and class sums.  Every border node is pointed at its root
// (find with full compression; no unions run any more), and the partial
// features (and minimum key) of every non-root node are added into its root.
// To keep the number of global atomics on the accumulators of components
// spanning many tiles (the exterior, percolating clusters) small, a workgroup
// first merges the contributions of the nodes of a group of consecutive tiles
// in an LDS hash table keyed by root and issues one set of atomics per root
// per flush.

constexpr int RH_CAP = 1024;     // LDS hash slots (power of two)
constexpr int RH_BITS = 10;      // log2(RH_CAP)
static_assert(1 << RH_BITS == RH_CAP, "hash width");
// tiles per workgroup: larger groups send fewer atomics to the roots of
// components that span many tiles (the exterior above all), but a grid of
// fewer workgroups than compute units leaves the chip idle.  Tiles of more
// than 4096 pixels of a single image take 128 per group where that still
// gives 256 groups, else 64 (measured: 16384^2 structured images 45 -> 32 us
// with 128; 8192^2 images 34 us with 64, 43 with 128, and more with 32; a
// batch of small images, whose exteriors are many roots, +0.5 % with 128).
template <class T>
inline int rh_group(int64_t tiles, bool one_image) {
  int g = T::RHT;
  if (T::RHT_AUTO)
    while (g > 64 && (!one_image || (tiles + g - 1) / g < 256)) g >>= 1;
  return g;
}
constexpr int RH_T = 512;        // threads: finds of many nodes in flight at once
constexpr int RH_EMPTY = -1;

struct RootAcc {
  int32_t key, minkey;
  int32_t xmin, xmax, ymin, ymax;
  u64 S, Sx, Sy;
};

__device__ inline void rootacc_clear(RootAcc& a) {
  a.key = RH_EMPTY;
  a.minkey = 0x7FFFFFFF;
  a.xmin = 0x7FFFFFFF;
  a.xmax = -1;
  a.ymin = 0x7FFFFFFF;
  a.ymax = -1;
  a.S = a.Sx = a.Sy = 0;
}

template <class T, class Src>
__global__ void __launch_bounds__(RH_T) k_reduce_roots(Src src, Work wk, int64_t tiles) {
  constexpr int RHT = T::RHT;  // the largest group
  static_assert(RHT <= 256 && (RHT & (RHT - 1)) == 0, "one wave scans the group, 64 tiles at a time");
  __shared__ RootAcc tab[RH_CAP];
  __shared__ int pre[RHT + 1];
  __shared__ int64_t tbase[RHT];
  __shared__ int32_t text[RHT];  // exterior node of the tile's image
  __shared__ int used;
  const int tid = threadIdx.x;
  const int G = wk.rh_group;  // this launch's group: a power of two <= RHT
  const int64_t t0 = (int64_t)blockIdx.x * G;
  const int ntl = tiles - t0 < G ? (int)(tiles - t0) : G;
  for (int i = tid; i < RH_CAP; i += RH_T) rootacc_clear(tab[i]);
  if (tid < 64) {  // node counts of the group's tiles -> exclusive prefix
    int carry = 0;
    for (int b = 0; b < G; b += 64) {
      const int k = b + tid;
      int c = 0;
      if (k < ntl) {
        const int64_t gt = t0 + k;
        const ImgDesc& d = src.by_tile(gt);
        c = src.ok(d) ? wk.nbt[gt] : 0;
        tbase[k] = tile_node_base<T>(d, gt - d.tile0);
        text[k] = (int32_t)d.node0;
      }
      int inc = c;
      for (int dl = 1; dl < 64; dl <<= 1) {
        int t = __shfl_up(inc, dl, 64);
        if (tid >= dl) inc += t;
      }
      if (k < G) pre[k] = carry + inc - c;
      if (k == G - 1) pre[G] = carry + inc;
      carry += __shfl(inc, 63, 64);
    }
  }
  if (tid == 0) used = 0;
  __syncthreads();
  const int total = pre[G];
  // the group's nodes as one list, RH_T at a time
  for (int base = 0; base < total; base += RH_T) {
    const int i = base + tid;
    if (i < total) {
      // the tile holding the group's i-th node: the last with pre <= i
      int k = 0;
      for (int half = G / 2; half >= 1; half >>= 1)
        if (k + half < G && pre[k + half] <= i) k += half;
      const int node = (int)(tbase[k] + (i - pre[k]));
      const Feature f = wk.gacc[node];
      const int32_t key = wk.gkey[node];
      const int r = gfind(wk.gpar, node);  // leaves gpar[node] == r
      if (r != node) {
        uint32_t hsh = ((uint32_t)r * 2654435761u) >> (32 - RH_BITS);
        int slot = (int)hsh;
        for (;;) {
          int k2 = atomicCAS(&tab[slot].key, RH_EMPTY, r);
          if (k2 == RH_EMPTY) {
            atomicAdd(&used, 1);
            break;
          }
          if (k2 == r) break;
          slot = (slot + 1) & (RH_CAP - 1);
        }
        RootAcc& a = tab[slot];
        atomicMin(&a.minkey, key);
        atomicMin(&a.xmin, f.xmin);
        atomicMax(&a.xmax, f.xmax);
        atomicMin(&a.ymin, f.ymin);
        atomicMax(&a.ymax, f.ymax);
        atomicAdd(&a.S, (u64)f.S);
        atomicAdd(&a.Sx, (u64)f.Sx);
        atomicAdd(&a.Sy, (u64)f.Sy);
      }
    }
    __syncthreads();
    // flush when another chunk might not fit, and at the end; every thread
    // reads the count before any thread inserts again
    const bool flush = used > RH_CAP - RH_T || base + RH_T >= total;
    __syncthreads();
    if (flush) {
      for (int j = tid; j < RH_CAP; j += RH_T) {
        RootAcc& a = tab[j];
        if (a.key == RH_EMPTY) continue;
        int r = a.key;
        // an exterior is the first node of its image's block, before all
        // of its tiles' nodes: compare with the one of the last tile whose
        // exterior is at or before r (no minimum key: the exterior's id is 0)
        int lo = 0, hi = ntl - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (text[mid] <= r) lo = mid;
          else hi = mid - 1;
        }
        Feature* g;
        if (text[lo] == r) {
          g = &wk.gacc[r + 1 + (int)(blockIdx.x % EXT_REP)];
        } else {
          atomicMin(&wk.gminkey[r], a.minkey);
          g = &wk.gacc[r];
        }
        atomicMin(&g->xmin, a.xmin);
        atomicMax(&g->xmax, a.xmax);
        atomicMin(&g->ymin, a.ymin);
        atomicMax(&g->ymax, a.ymax);
        atomicAdd(reinterpret_cast<unsigned long long*>(&g->S), (unsigned long long)a.S);
        atomicAdd(reinterpret_cast<unsigned long long*>(&g->Sx), (unsigned long long)a.Sx);
        atomicAdd(reinterpret_cast<unsigned long long*>(&g->Sy), (unsigned long long)a.Sy);
        rootacc_clear(a);
      }
      if (tid == 0) used = 0;
      __syncthreads();
    }
  }
}

// The same work without the LDS table: every non-root node adds its partial
// directly into its root with global atomics (one wave per tile).
// Cheaper when components rarely span tiles; contended on giant ones.
template <class T, class Src>
__global__ void __launch_bounds__(64) k_reduce_direct(Src src, Work wk) {
  const int64_t gt = blockIdx.x;
  const ImgDesc& d = src.by_tile(gt);
  if (!src.ok(d)) return;
  const int64_t nbase = tile_node_base<T>(d, gt - d.tile0);
  const int nb = wk.nbt[gt];
  for (int i = threadIdx.x; i < nb; i += 64) {
    int node = (int)(nbase + i);
    int r = gfind(wk.gpar, node);  // leaves gpar[node] == r
    if (r == node) continue;
    Feature* g;
    if (r == (int)d.node0) {  // the exterior: one of its accumulators
      g = &wk.gacc[r + 1 + (int)(gt % EXT_REP)];
    } else {
      atomicMin(&wk.gminkey[r], wk.gkey[node]);
      g = &wk.gacc[r];
    }
    Feature f = wk.gacc[node];
    atomicMin(&g->xmin, f.xmin);
    atomicMax(&g->xmax, f.xmax);
    atomicMin(&g->ymin, f.ymin);
    atomicMax(&g->ymax, f.ymax);
    atomicAdd(reinterpret_cast<unsigned long long*>(&g->S), (unsigned long long)f.S);
    atomicAdd(reinterpret_cast<unsigned long long*>(&g->Sx), (unsigned long long)f.Sx);
    atomicAdd(reinterpret_cast<unsigned long long*>(&g->Sy), (unsigned long long)f.Sy);
  }
}

// ---------------------------------------------------------------------------
// K4: leaders (node holding the component's first pixel) and their ranks

template <class T, class Src>
__global__ void __launch_bounds__(64) k_leaders(Src src, Work wk) {
  __shared__ u16 pre[T::BCAP + 1];
  __shared__ u32 first[T::TH];
  __shared__ u32 cnt[T::TH];
  __shared__ int32_t rl[T::BCAP];  // the node's root, HI set when the node leads its component
  __shared__ int32_t gr[T::BCAP];  // the node's row and rank from K1
  const int64_t gt = blockIdx.x;
  const ImgDesc& d = src.by_tile(gt);
  if (!src.ok(d)) return;
  const int64_t lt = gt - d.tile0;
  const int tx = (int)(lt % d.ntx), ty = (int)(lt / d.ntx);
  const int y0 = ty * T::TH;
  const int th = d.h - y0 < T::TH ? d.h - y0 : T::TH;
  const int64_t nbase = tile_node_base<T>(d, lt);
  const int nb = wk.nbt[gt];
  const int lane = threadIdx.x;
  for (int ly = lane; ly < T::TH; ly += 64) {
    first[ly] = 0xFFFFu;
    cnt[ly] = 0;
  }
  __syncthreads();
  u32 carry = 0;
  for (int base = 0; base < nb; base += 64) {
    int i = base + lane;
    bool lead = false;
    if (i < nb) {
      int node = (int)(nbase + i);
      int r = wk.gpar[node];
      const bool ext = r == (int)d.node0;
      const int32_t mk = ext ? 0 : wk.gminkey[r];
      lead = !ext && mk == wk.gkey[node];
      if (!ext) {  // the (row, tile column) cell of the component's first pixel, for k_border_canon
        const int y = mk / d.w, x = mk - y * d.w;
        wk.ncanon[node] = y * d.ntx + x / T::TW;
      }
      const int g = wk.grank[node];
      int ly = (g >> 16) & 63;
      rl[i] = lead ? (int)((u32)r | HI) : r;
      gr[i] = g;
      atomicMin(&first[ly], (u32)i);
      if (lead) atomicAdd(&cnt[ly], 1u);
    }
    u64 bal = __ballot(lead);
    if (i < nb) pre[i] = (u16)(carry + popc64(bal & low_mask(lane)));
    carry += (u32)popc64(bal);
  }
  if (lane == 0) pre[nb] = (u16)carry;
  __syncthreads();
  for (int i = lane; i < nb; i += 64) {  // from LDS: no second round of dependent loads
    int node = (int)(nbase + i);
    int g = gr[i];
    int ly = (g >> 16) & 63;
    const int rv = rl[i];
    const bool lead = rv < 0;
    const int r = rv & 0x7FFFFFFF;
    int rank = (g & 0xFFFF) + (int)pre[i] - (int)pre[first[ly]];
    wk.grank[node] = rank | (ly << 16) | (lead ? (int)HI : 0);
    if (lead) wk.rcanon[r] = rank;  // the component's rank in its first pixel's cell
  }
  for (int ly = lane; ly < th; ly += 64) {
    if (cnt[ly]) wk.cgrid[d.c0 + (int64_t)(y0 + ly) * d.ntx + tx] += (int)cnt[ly];
  }
}

// ---------------------------------------------------------------------------
// scan of the count grid, per image: base = 1 + exclusive prefix

__device__ inline u32 block_excl_scan(u32 v, u32* wsum, u32& total) {
  // each wave scans its 64 values in registers; the waves' totals go
  // through LDS (two barriers; wsum holds SCAN_T / 64 entries)
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  u32 inc = v;
  for (int dl = 1; dl < 64; dl <<= 1) {
    u32 x = __shfl_up(inc, dl, 64);
    if (lane >= dl) inc += x;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  u32 before = 0, all = 0;
  for (int k = 0; k < SCAN_T / 64; k++) {
    const u32 s = wsum[k];
    before += k < wv ? s : 0u;
    all += s;
  }
  total = all;
  __syncthreads();  // wsum is free for the next call
  return before + inc - v;
}

template <class Src>
__global__ void __launch_bounds__(SCAN_T) k_scan_reduce(Src src, Work wk) {
  __shared__ u32 tmp[SCAN_T / 64];
  const int64_t gb = blockIdx.x;
  const ImgDesc& d = src.by_block(gb);
  if (!src.ok(d)) return;
  const int64_t n = (int64_t)d.h * d.ntx;
  const int64_t b0 = (gb - d.blk0) * SCAN_B;
  u32 v = 0;
  for (int k = 0; k < 4; k++) {
    int64_t e = b0 + threadIdx.x * 4 + k;
    if (e < n) v += (u32)wk.cgrid[d.c0 + e];
  }
  u32 tot;
  block_excl_scan(v, tmp, tot);
  if (threadIdx.x == 0) wk.bsum[gb] = (int32_t)tot;
}

template <class Src>
__global__ void __launch_bounds__(SCAN_T) k_scan_apply(Src src, Work wk) {
  __shared__ u32 tmp[SCAN_T / 64];
  const int64_t gb = blockIdx.x;
  const ImgDesc& d = src.by_block(gb);
  if (!src.ok(d)) return;
  const int64_t n = (int64_t)d.h * d.ntx;
  const int64_t b0 = (gb - d.blk0) * SCAN_B;
  u32 v[4];
  u32 sum = 0;
  for (int k = 0; k < 4; k++) {
    int64_t e = b0 + threadIdx.x * 4 + k;
    v[k] = e < n ? (u32)wk.cgrid[d.c0 + e] : 0u;
    sum += v[k];
  }
  // ids before this block: the totals of the image's earlier blocks (a few
  // thousand at most per image, summed here rather than scanned by a kernel
  // of their own)
  u32 part = 0;
  for (int64_t b = d.blk0 + threadIdx.x; b < gb; b += SCAN_T) part += (u32)wk.bsum[b];
  u32 before;
  (void)block_excl_scan(part, tmp, before);
  u32 tot;
  u32 ex = block_excl_scan(sum, tmp, tot) + before + 1u;
  for (int k = 0; k < 4; k++) {
    int64_t e = b0 + threadIdx.x * 4 + k;
    if (e < n) wk.cgrid[d.c0 + e] = (int32_t)ex;
    ex += v[k];
  }
  // the image's last block knows the number of labels (exterior included)
  if (threadIdx.x == 0 && gb == d.blk0 + d.nblk - 1 && d.counts) d.counts[0] = 1 + (int64_t)before + (int64_t)tot;
}

// ---------------------------------------------------------------------------
// K5: the canonical id of every border node (its component's), and the
// tables of the components that cross tiles, written by the node holding the
// component's first pixel.  The id is the scanned base of the (row, tile
// column) cell of the component's first pixel (the minimum key at the root)
// plus the component's rank among the components starting in that cell,
// which k_leaders left at the root.

template <class T, class Src>
__global__ void __launch_bounds__(64) k_border_canon(Src src, Work wk) {
  __shared__ int32_t cl[T::BCAP];  // canonical id by node slot
  const int64_t gt = blockIdx.x;
  const ImgDesc& d = src.by_tile(gt);
  if (!src.ok(d)) return;
  const int64_t lt = gt - d.tile0;
  const int64_t nbase = tile_node_base<T>(d, lt);
  const int nb = wk.nbt[gt];
  // node slot of each row's last pixel (entries past the tile's rows unused)
  const u16 rslot = wk.bidx_v[(gt * 2 + 1) * T::TH + (threadIdx.x < T::TH ? threadIdx.x : 0)];
  if (lt == 0 && threadIdx.x == 0) {
    if (d.feat) {
      Feature e = wk.gacc[d.node0];
      for (int k = 1; k <= EXT_REP; k++) {
        const Feature f = wk.gacc[d.node0 + k];
        e.xmin = f.xmin < e.xmin ? f.xmin : e.xmin;
        e.xmax = f.xmax > e.xmax ? f.xmax : e.xmax;
        e.ymin = f.ymin < e.ymin ? f.ymin : e.ymin;
        e.ymax = f.ymax > e.ymax ? f.ymax : e.ymax;
        e.S += f.S;
        e.Sx += f.Sx;
        e.Sy += f.Sy;
      }
      d.feat[0] = e;
    }
    if (d.parent) d.parent[0] = -1;
    if (d.color) d.color[0] = 0;
  }
  for (int i = threadIdx.x; i < nb; i += 64) {
    const int node = (int)(nbase + i);
    const int r = wk.gpar[node];
    const int g = wk.grank[node];
    const int cell = wk.ncanon[node];  // k_leaders left the cell of the component's first pixel here
    int32_t canon = 0;
    if (r != (int)d.node0) canon = wk.cgrid[d.c0 + cell] + wk.rcanon[r];
    wk.ncanon[node] = canon;
    cl[i] = canon;
    if ((g & (int)HI) && d.feat && canon < d.cap) d.feat[canon] = wk.gacc[r];
  }
  // the ids at the right column, row by row: the parents of the components
  // of the right neighbour whose first pixel is in its column 0
  __syncthreads();
  const int y0 = (int)(lt / d.ntx) * T::TH;
  const int th = d.h - y0 < T::TH ? d.h - y0 : T::TH;
  if ((int)threadIdx.x < th) wk.rcol[gt * T::TH + threadIdx.x] = cl[rslot];
}

// ---------------------------------------------------------------------------
// K6: relabel the tile, write labels and the tables of the components it
// owns.  Works from the tile state K1 left (no image reload, no union-find).

template <class T>
struct EmitSmem {
  u64 bits[T::NW];
  u64 st[T::NW];       // run starts
  u64 rootm[T::NW];    // roots
  u64 broot[T::NW];    // roots of components touching the tile border
  u64 lmask[T::NW];    // roots that hold their component's first pixel
  u16 spre[T::NW];     // run starts before word (tile raster order)
  u16 bpre[T::NW];     // border roots before word
  u16 ipre[T::NW];     // interior roots before word
  struct {
    u16 ordr[T::N];  // root ordinal by run rank
    // interior root nb + i: its position (row * TW + column), from step 5 on
    // row << 8 | rank among the row's leaders.  A tile has fewer than N / 2
    // interior components: their first pixels
    // (the roots) lie off the tile's edge rows and columns, and no two are
    // next to each other in a row (if (x, y) and (x + 1, y) both were
    // first pixels, (x + 1, y - 1) has the colour of (x, y), else it would
    // precede (x + 1, y) in its component; if that colour is the
    // 8-adjacent one it joins (x, y) from an earlier row, else (x, y - 1)
    // has the other colour, which then joins (x + 1, y) diagonally from an
    // earlier row)
    u16 ipos[T::N / 2];
  } rt;
  int32_t bcanon[T::BCAP];  // canonical id of border root ordinal o (o < nb); HI: holds its first pixel
  int32_t rowbase[T::TH];  // first canonical id of the row's components starting here
  int32_t lcanon[T::TH];   // canonical id of the pixel left of the tile, per row
  int nb, nint, nruns, euler;
};

// canonical id of root ordinal o; the interior table holds positions
// (POS) or, once step 5 has converted it, row << 8 | rank among the row's
// leaders
template <bool POS, class T>
__device__ inline int32_t canon_of(const EmitSmem<T>& s, int o) {
  // both tables are read (no divergent branch), the right one selected
  const int nb = s.nb;
  const bool border = o < nb;
  const int32_t cb = s.bcanon[border ? o : 0] & ~(int32_t)HI;
  const u32 v = s.rt.ipos[border ? 0 : o - nb];
  int32_t ci;
  if constexpr (POS) {
    // the row's base plus the leaders before the root in its row
    const int ly = (int)(v / T::TW), x = (int)(v % T::TW), j = x >> 6;
    int rank = popc64(s.lmask[ly * T::WPR + j] & low_mask(x & 63));
#pragma unroll
    for (int jj = 0; jj < T::WPR - 1; jj++)
      if (jj < j) rank += popc64(s.lmask[ly * T::WPR + jj]);
    ci = s.rowbase[ly] + (int32_t)rank;
  } else {
    ci = s.rowbase[v >> 8] + (int32_t)(v & 0xFFu);
  }
  return border ? cb : ci;
}

template <class T>
__device__ inline int run_rank(const EmitSmem<T>& s, int ly, int x) {  // run holding pixel (ly, x)
  int wd = ly * T::WPR + (x >> 6);
  return s.spre[wd] + popc64(s.st[wd] & (~0ull >> (63 - (x & 63)))) - 1;
}

// Segments of one 16-pixel chunk: calls f(run_rank, seg_begin, seg_end).
template <class T, class Fn>
__device__ inline void for_runs(const EmitSmem<T>& s, int ly, int cc, int tw, Fn f) {
  int cs = cc * 16;
  if (cs >= tw) return;
  int ce = cs + 16 < tw ? cs + 16 : tw;
  int j = cc >> 2, sh = (cc & 3) * 16;
  u32 m = ((u32)(s.st[ly * T::WPR + j] >> sh) & 0xFFFFu) & ~1u;
  int rank = run_rank(s, ly, cs);
  int x = cs;
  for (;;) {
    int nx = m ? cs + ctz32(m) : ce;
    f(rank, x, nx);
    if (!m) break;
    m &= m - 1;
    rank++;
    x = nx;
  }
}

template <class T, class Src>
__global__ void __launch_bounds__(T::NT) k_tile_emit(Src src, Work wk) {
  __shared__ EmitSmem<T> s;
  __shared__ AccP iacc[T::CAPI];
  const int64_t gt = blockIdx.x;
  const ImgDesc& d = src.by_tile(gt);
  if (!src.ok(d)) return;
  const int64_t lt = gt - d.tile0;
  const int tx = (int)(lt % d.ntx), ty = (int)(lt / d.ntx);
  const int x0 = tx * T::TW, y0 = ty * T::TH;
  const int tw = d.w - x0 < T::TW ? d.w - x0 : T::TW;
  const int th = d.h - y0 < T::TH ? d.h - y0 : T::TH;
  const int tid = threadIdx.x;
  const int64_t nbase = tile_node_base<T>(d, lt);
  // the tile's kind and its first node's id and rank, in one round trip
  // (relaxed atomic loads are issued where they are written; plain loads
  // would be moved into the branches that use them, one after the other)
  const int info = ld_now(&wk.tinfo[gt]);
  const int nbt = ld_now(&wk.nbt[gt]);
  const int32_t canon0 = ld_now(&wk.ncanon[nbase]);
  const int grank0 = ld_now(&wk.grank[nbase]);

  if (info & 3) {
    // one-colour tile: its single component is border node slot 0
    const int col = (info & 3) - 1;
    const int32_t canon = canon0;
    if (tid == 0 && (grank0 & (int)HI)) {  // the component starts here
      if (canon < d.cap) {
        if (d.color) d.color[canon] = (u8)col;
        if (d.parent) d.parent[canon] = tx > 0 ? wk.rcol[(gt - 1) * T::TH] : 0;
      }
      if (d.counts)
        atomicAdd(reinterpret_cast<unsigned long long*>(&d.counts[1]), (unsigned long long)(int64_t)(col ? 1 : -1));
    }
    if (d.labels) {
      const bool vec = (d.flags & DF_VEC_LAB) != 0;
      for (int q = tid; q < T::TH * (T::TW / 4); q += T::NT) {
        int ly = q / (T::TW / 4), x = (q % (T::TW / 4)) * 4;
        if (ly >= th || x >= tw) continue;
        int32_t* dst = d.labels + (int64_t)(y0 + ly) * d.w + x0 + x;
        if (vec && x + 4 <= tw) {
          store_labels4(dst, canon, canon, canon, canon);
        } else {
          int n = tw - x < 4 ? tw - x : 4;
          for (int k = 0; k < n; k++) dst[k] = canon;
        }
      }
    }
    return;
  }

  // 1. tile state, root ordinals of the runs, row bases; canonical ids of the
  // border roots (HI marks the ones holding their component's first pixel);
  // the first pass of interior accumulators cleared.  All of it is requested
  // before any is used (one-colour tiles read none of it).
  const u64* ts = wk.tstate + gt * 3 * T::NW;
  u64 tsv[(3 * T::NW + T::NT - 1) / T::NT];
#pragma unroll
  for (int k = 0; k < (3 * T::NW + T::NT - 1) / T::NT; k++) {
    int i = tid + k * T::NT;
    tsv[k] = i < 3 * T::NW ? ts[i] : 0ull;
  }
  const int32_t rowb = tid < th ? wk.cgrid[d.c0 + (int64_t)(y0 + tid) * d.ntx + tx] : 0;
  // canonical id at the left neighbour's right column, per row (parents of
  // components whose first pixel is in column 0; 0, the exterior, at the
  // image's left edge)
  const bool has_left = tid < th && tx > 0;
  const int32_t lcv = has_left ? wk.rcol[(gt - 1) * T::TH + tid] : 0;
  const u32 ord2 = reinterpret_cast<const u32*>(wk.tord + gt * T::N)[tid < T::N / 2 ? tid : 0];
  const int bslot = tid < T::BCAP ? tid : 0;
  const int32_t bcan = wk.ncanon[nbase + bslot];
  const int bgr = wk.grank[nbase + bslot];
  const int nruns = info >> 2;
#pragma unroll
  for (int k = 0; k < (3 * T::NW + T::NT - 1) / T::NT; k++) {
    int i = tid + k * T::NT;
    if (i < 3 * T::NW) {
      int kk = i / T::NW, wd = i % T::NW;
      if (kk == 0) s.bits[wd] = tsv[k];
      else if (kk == 1) s.rootm[wd] = tsv[k];
      else s.broot[wd] = tsv[k];
    }
  }
  const u16* to = wk.tord + gt * T::N;
  if (2 * tid < nruns && tid < T::N / 2) {
    s.rt.ordr[2 * tid] = (u16)(ord2 & 0xFFFFu);
    if (2 * tid + 1 < nruns) s.rt.ordr[2 * tid + 1] = (u16)(ord2 >> 16);
  }
  for (int r = 2 * T::NT + tid; r < nruns; r += T::NT) s.rt.ordr[r] = to[r];
  if (tid < th) s.rowbase[tid] = rowb;
  if (tid < nbt && tid < T::BCAP) s.bcanon[tid] = bcan | (bgr & (int)HI);
  for (int bi = T::NT + tid; bi < nbt; bi += T::NT) s.bcanon[bi] = wk.ncanon[nbase + bi] | (wk.grank[nbase + bi] & (int)HI);
  if (tid == 0) s.euler = 0;
  for (int i = tid; i < T::CAPI; i += T::NT) acc_init(iacc[i]);
  __syncthreads();

  // 2. a word per lane, one wave per 64 words: run starts; exclusive prefix
  // counts over words of border roots, interior roots and run starts
  // (each wave adds the counts of the words before its own, which it sums
  // itself: no wave waits for another); leaders (roots holding their
  // component's first pixel: every interior root, and the border roots
  // whose HI mark is set)
  {
    constexpr int NWV = (T::NW + 63) / 64;  // waves at work
    static_assert(NWV * 64 <= T::NT, "a wave per 64 words");
    const int wv = tid >> 6, lane = tid & 63;
    // the counts of one word: border roots | interior roots << 16, run starts
    auto counts = [&](int wd, u64& e, u64& rm, u64& bm) {
      const int ly = wd / T::WPR, j = wd % T::WPR;
      const u64 b = s.bits[wd];
      const u64 carry = j ? (s.bits[wd - 1] >> 63) : (~b & 1ull);
      e = ly < th ? (b ^ ((b << 1) | carry)) & valid_mask(j, tw) : 0ull;
      rm = s.rootm[wd];
      bm = s.broot[wd];
    };
    if (wv < NWV) {
      // counts of the words before this wave's
      u32 cb = 0, ci = 0, cs = 0;
      for (int wd = lane; wd < 64 * wv; wd += 64) {
        u64 e, rm, bm;
        counts(wd, e, rm, bm);
        cb += (u32)popc64(bm);
        ci += (u32)popc64(rm & ~bm);
        cs += (u32)popc64(e);
      }
      if (wv > 0) {
        cb = (u32)wave_sum((int)cb);
        ci = (u32)wave_sum((int)ci);
        cs = (u32)wave_sum((int)cs);
      }
      const int wd = 64 * wv + lane;
      u64 e = 0, rm = 0, bm = 0;
      if (wd < T::NW) counts(wd, e, rm, bm);
      const u32 v = (u32)popc64(bm) | ((u32)popc64(rm & ~bm) << 16);  // both <= 4096 per 64 words
      const u32 vs = (u32)popc64(e);
      u32 inc = v, incs = vs;
      for (int dl = 1; dl < 64; dl <<= 1) {
        u32 t = __shfl_up(inc, dl, 64);
        u32 t2 = __shfl_up(incs, dl, 64);
        if (lane >= dl) {
          inc += t;
          incs += t2;
        }
      }
      if (wd < T::NW) {
        const u32 exc = inc - v;
        const int bp = (int)(cb + (exc & 0xFFFFu));
        s.bpre[wd] = (u16)bp;
        s.ipre[wd] = (u16)(ci + (exc >> 16));
        s.spre[wd] = (u16)(cs + incs - vs);
        s.st[wd] = e;
        u64 lead = rm & ~bm;
        // (reads only: the mark stays in the table and is masked where the
        // ids are read, so that the reads of a word's roots overlap)
        int bi = bp;
        for (u64 m = bm; m; m &= m - 1, bi++) {
          if (s.bcanon[bi] & (int32_t)HI) lead |= m & (~m + 1ull);
        }
        s.lmask[wd] = lead;
      }
      if (wv == NWV - 1 && lane == 63) {
        s.nb = (int)(cb + (inc & 0xFFFFu));
        s.nint = (int)(ci + (inc >> 16));
        s.nruns = (int)(cs + incs);
      }
    }
  }
  __syncthreads();

  // 3. per chunk: positions of the interior roots, the Euler number over
  // the components that start here, and the features of interior components
  // (first CAPI of them)
  const int nb = s.nb;
  const int nint = s.nint;
  {
    int e_local = 0;
    for (int c = tid; c < T::NCH; c += T::NT) {
      const int ly = c / T::CPR, cc = c % T::CPR;
      const int j = cc >> 2, sh = (cc & 3) * 16;
      const int wd = ly * T::WPR + j;
      const u32 lm = reinterpret_cast<const u16*>(s.lmask)[c];
      const u32 b16 = reinterpret_cast<const u16*>(s.bits)[c];
      e_local += popc64(lm & b16) - popc64(lm & ~b16 & 0xFFFFu);
      const u64 imw = s.rootm[wd] & ~s.broot[wd];
      u32 im = (u32)(imw >> sh) & 0xFFFFu;
      for (int ii = s.ipre[wd] + popc64(imw & low_mask(sh)); im; im &= im - 1, ii++) {
        if (ii < T::N / 2) s.rt.ipos[ii] = (u16)(ly * T::TW + j * 64 + sh + ctz32(im));
      }
      if (ly >= th) continue;
      RowSum rs;
      rs.o = -1;
      for_runs<T>(s, ly, cc, tw, [&](int rank, int a, int b) {
        const int o = (int)s.rt.ordr[rank] - nb;
        if (o >= 0 && o < T::CAPI) rowsum_add(rs, iacc, o, ly, a, b);
      });
      rowsum_flush(rs, iacc, ly);
    }
    e_local = wave_sum(e_local);
    if ((tid & 63) == 0 && e_local) atomicAdd(&s.euler, e_local);
  }
  __syncthreads();
  if (tid == 0 && s.euler != 0 && d.counts)
    atomicAdd(reinterpret_cast<unsigned long long*>(&d.counts[1]), (unsigned long long)(int64_t)s.euler);

  // 4. tables of interior components (colour, parent, features), CAPI at a
  // time: the first pass was accumulated in step 3
  for (int k0 = 0; k0 < nint; k0 += T::CAPI) {
    if (k0 > 0) {
      for (int i = tid; i < T::CAPI; i += T::NT) acc_init(iacc[i]);
      __syncthreads();
      for (int c = tid; c < T::NCH; c += T::NT) {
        int ly = c / T::CPR, cc = c % T::CPR;
        if (ly >= th) continue;
        RowSum rs;
        rs.o = -1;
        for_runs<T>(s, ly, cc, tw, [&](int rank, int a, int b) {
          int o = (int)s.rt.ordr[rank] - nb - k0;
          if (o >= 0 && o < T::CAPI) rowsum_add(rs, iacc, o, ly, a, b);
        });
        rowsum_flush(rs, iacc, ly);
      }
      __syncthreads();
    }
    // one thread per interior component (not one per chunk: a chunk's
    // components would be worked off one after another by its lane)
    const int kn = nint - k0 < T::CAPI ? nint - k0 : T::CAPI;
    for (int o = tid; o < kn; o += T::NT) {
      const int ii = k0 + o;
      const u32 p = s.rt.ipos[ii];
      const int ly = (int)(p / T::TW), xk = (int)(p % T::TW);
      const int wd = ly * T::WPR + (xk >> 6);
      const int32_t canon = canon_of<true>(s, nb + ii);
      if (canon >= d.cap) continue;
      if (d.feat) d.feat[canon] = acc_abs(iacc[o], ly, x0, y0);
      if (d.color) d.color[canon] = (u8)((s.bits[wd] >> (xk & 63)) & 1ull);
      if (d.parent) d.parent[canon] = canon_of<true>(s, s.rt.ordr[run_rank(s, ly, xk - 1)]);  // interior: x > 0
    }
    if (k0 + T::CAPI < nint) __syncthreads();  // the accumulators are cleared next
  }

  // 5. the interior table from positions to row << 8 | rank among the row's
  // leaders (cheaper to map for the many lookups of steps 6 and 7); the left
  // neighbour's ids where step 6 reads them
  __syncthreads();
  for (int ii = tid; ii < nint; ii += T::NT) {
    const u32 v = s.rt.ipos[ii];
    const int ly = (int)(v / T::TW), x = (int)(v % T::TW), j = x >> 6;
    int rank = popc64(s.lmask[ly * T::WPR + j] & low_mask(x & 63));
#pragma unroll
    for (int jj = 0; jj < T::WPR - 1; jj++)
      if (jj < j) rank += popc64(s.lmask[ly * T::WPR + jj]);
    s.rt.ipos[ii] = (u16)((ly << 8) | rank);
  }
  if (tid < th) s.lcanon[tid] = lcv;
  __syncthreads();

  // 6. colour / parent of border components whose first pixel is here
  for (int c = tid; c < T::NCH; c += T::NT) {
    int ly = c / T::CPR, cc = c % T::CPR;
    int j = cc >> 2, sh = (cc & 3) * 16;
    int wd = ly * T::WPR + j;
    const u64 bmw = s.broot[wd];
    for (u32 bl = (u32)((bmw & s.lmask[wd]) >> sh) & 0xFFFFu; bl; bl &= bl - 1) {
      int k = sh + ctz32(bl);
      int32_t canon = s.bcanon[s.bpre[wd] + popc64(bmw & low_mask(k))] & ~(int32_t)HI;
      if (canon >= d.cap) continue;
      if (d.color) d.color[canon] = (u8)((s.bits[wd] >> k) & 1ull);
      if (d.parent) {
        int x = j * 64 + k;
        int32_t pc;
        if (x == 0) pc = s.lcanon[ly];  // 0 (exterior) at the image's left edge
        else pc = canon_of<false>(s, s.rt.ordr[run_rank(s, ly, x - 1)]);
        d.parent[canon] = pc;
      }
    }
  }

  // 7. label image, four pixels per thread (the canonical id of each run
  // the four pixels touch, taken from the root ordinal once per run)
  if (d.labels) {
    const bool vec = (d.flags & DF_VEC_LAB) != 0;
    for (int q = tid; q < T::TH * (T::TW / 4); q += T::NT) {
      int ly = q / (T::TW / 4), x = (q % (T::TW / 4)) * 4;
      if (ly >= th || x >= tw) continue;
      const int r0 = run_rank(s, ly, x);
      const u32 sw = (u32)(s.st[ly * T::WPR + (x >> 6)] >> (x & 63));
      const int r1 = r0 + (int)((sw >> 1) & 1u);
      const int r2 = r1 + (int)((sw >> 2) & 1u);
      const int r3 = r2 + (int)((sw >> 3) & 1u);
      int32_t lab[4];
      lab[0] = canon_of<false>(s, s.rt.ordr[r0]);
      lab[1] = r1 == r0 ? lab[0] : canon_of<false>(s, s.rt.ordr[r1]);
      lab[2] = r2 == r1 ? lab[1] : canon_of<false>(s, s.rt.ordr[r2]);
      lab[3] = r3 == r2 ? lab[2] : canon_of<false>(s, s.rt.ordr[r3]);
      int32_t* dst = d.labels + (int64_t)(y0 + ly) * d.w + x0 + x;
      if (vec && x + 4 <= tw) {
        store_labels4(dst, lab[0], lab[1], lab[2], lab[3]);
      } else {
        int n = tw - x < 4 ? tw - x : 4;
        for (int k = 0; k < n; k++) dst[k] = lab[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host side: workspace layout and the launch sequence

struct Layout {
  int64_t tiles, nodes, cells, blocks;
  size_t off_gpar, off_gkey, off_gminkey, off_grank, off_rcanon, off_ncanon, off_gacc, off_nbt;
  size_t off_bidxh, off_bidxv, off_bitsh, off_bitslr;
  size_t off_cgrid, off_bsum, off_tinfo, off_tstate, off_tord, off_rcol, bytes;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

template <class T>
inline Layout make_layout(int64_t tiles, int64_t nodes, int64_t cells, int64_t blocks) {
  Layout L;
  L.tiles = tiles;
  L.nodes = nodes;
  L.cells = cells;
  L.blocks = blocks;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_gpar = take(4 * (size_t)nodes);
  L.off_gkey = take(4 * (size_t)nodes);
  L.off_gminkey = take(4 * (size_t)nodes);
  L.off_grank = take(4 * (size_t)nodes);
  L.off_rcanon = take(4 * (size_t)nodes);
  L.off_ncanon = take(4 * (size_t)nodes);
  L.off_gacc = take(sizeof(Feature) * (size_t)nodes);
  L.off_nbt = take(4 * (size_t)tiles);
  L.off_bidxh = take(2 * 2 * (size_t)tiles * T::TW);
  L.off_bidxv = take(2 * 2 * (size_t)tiles * T::TH);
  L.off_bitsh = take(8 * 2 * (size_t)tiles * T::WPR);
  L.off_bitslr = take(16 * (size_t)tiles);
  L.off_cgrid = take(4 * (size_t)cells);
  L.off_bsum = take(4 * (size_t)blocks);
  L.off_tinfo = take(4 * (size_t)tiles);
  L.off_tstate = take(8 * 3 * (size_t)tiles * T::NW);
  L.off_tord = take(2 * (size_t)tiles * T::N);
  L.off_rcol = take(4 * (size_t)tiles * T::TH);
  L.bytes = o;
  return L;
}

inline Work make_work(const Layout& L, void* ws) {
  char* b = static_cast<char*>(ws);
  Work w;
  w.gpar = reinterpret_cast<int32_t*>(b + L.off_gpar);
  w.gkey = reinterpret_cast<int32_t*>(b + L.off_gkey);
  w.gminkey = reinterpret_cast<int32_t*>(b + L.off_gminkey);
  w.grank = reinterpret_cast<int32_t*>(b + L.off_grank);
  w.rcanon = reinterpret_cast<int32_t*>(b + L.off_rcanon);
  w.ncanon = reinterpret_cast<int32_t*>(b + L.off_ncanon);
  w.gacc = reinterpret_cast<Feature*>(b + L.off_gacc);
  w.nbt = reinterpret_cast<int32_t*>(b + L.off_nbt);
  w.bidx_h = reinterpret_cast<u16*>(b + L.off_bidxh);
  w.bidx_v = reinterpret_cast<u16*>(b + L.off_bidxv);
  w.bits_h = reinterpret_cast<u64*>(b + L.off_bitsh);
  w.bits_lr = reinterpret_cast<u64*>(b + L.off_bitslr);
  w.cgrid = reinterpret_cast<int32_t*>(b + L.off_cgrid);
  w.bsum = reinterpret_cast<int32_t*>(b + L.off_bsum);
  w.tinfo = reinterpret_cast<int32_t*>(b + L.off_tinfo);
  w.tstate = reinterpret_cast<u64*>(b + L.off_tstate);
  w.tord = reinterpret_cast<u16*>(b + L.off_tord);
  w.rcol = reinterpret_cast<int32_t*>(b + L.off_rcol);
  w.k1_stride = 1u;
  w.rh_group = 1;
  return w;
}

// per-image geometry; fills the derived fields of d given running offsets
template <class T>
inline void place_image(ImgDesc& d, int64_t& tiles, int64_t& nodes, int64_t& cells, int64_t& blocks,
                        int64_t& items, int64_t& supers) {
  d.ntx = (d.w + T::TW - 1) / T::TW;
  d.nty = (d.h + T::TH - 1) / T::TH;
  int64_t nt = (int64_t)d.ntx * d.nty;
  int64_t nc = (int64_t)d.h * d.ntx;
  d.nblk = (int32_t)((nc + SCAN_B - 1) / SCAN_B);
  d.tile0 = tiles;
  d.node0 = nodes;
  d.c0 = cells;
  d.blk0 = blocks;
  d.it0 = items;
  d.nit = merge_items<T>(d.w, d.h, d.ntx, d.nty);
  d.s0 = supers;
  supers += (int64_t)((d.ntx + T::SUP - 1) / T::SUP) * ((d.nty + T::SUP - 1) / T::SUP);
  tiles += nt;
  nodes += 1 + EXT_REP + nt * T::BCAP;
  cells += nc;
  blocks += d.nblk;
  items += d.nit;
}

// Stride of a scattered tile order: about 0.618 of the tile count (successive
// workgroups land far apart) and coprime to it (a permutation).
inline uint32_t scatter_stride(int64_t tiles) {
  if (tiles <= 2) return 1u;
  const uint64_t t = (uint64_t)tiles;
  uint64_t s = (uint64_t)((double)t * 0.6180339887) | 1u;
  auto gcd = [](uint64_t a, uint64_t b) {
    while (b) {
      uint64_t r = a % b;
      a = b;
      b = r;
    }
    return a;
  };
  while (gcd(s, t) != 1) s += 2;
  return (uint32_t)(s % t);
}

// Enqueue the whole path.  `L` provides launch(kernel, grid, block, args...)
// in stream order.  Every image's derived fields must come from place_image.
// HASH selects the root reduction: LDS hash per group of tiles, or direct
// global atomics per node.
template <class T, bool HASH, class Src, class Launcher>
inline void enqueue(Launcher& L, const Src& src, const Work& wk0, int64_t tiles, int64_t items, int64_t blocks,
                    int64_t supers) {
  // K1 takes the tiles of a single image in a scattered order: neighbouring
  // tiles tend to be of one kind (one-colour tiles, which only load, or
  // general tiles, which compute), and workgroups of both kinds resident
  // together overlap better than a run of either (measured: -12 % on K1 for
  // the structured 16384^2 images, no change on random ones; K6 gains
  // nothing; a batch of small images loses 2 % and keeps raster order).
  Work wk = wk0;
  if constexpr (std::is_same<Src, OneImage>::value) wk.k1_stride = scatter_stride(tiles);
  L.launch(k_tile_export<T, Src>, tiles, T::NT, src, wk);
  L.launch(k_seam_local<T, Src>, supers, sl_threads<T>(), src, wk);
  if (items > 0) L.launch(k_border_merge<T, Src>, (items + 255) / 256, 256, src, wk, items);
  if (HASH) {
    wk.rh_group = rh_group<T>(tiles, std::is_same<Src, OneImage>::value);
    L.launch(k_reduce_roots<T, Src>, (tiles + wk.rh_group - 1) / wk.rh_group, RH_T, src, wk, tiles);
  }
  else L.launch(k_reduce_direct<T, Src>, tiles, 64, src, wk);
  L.launch(k_leaders<T, Src>, tiles, 64, src, wk);
  L.launch(k_scan_reduce<Src>, blocks, SCAN_T, src, wk);
  L.launch(k_scan_apply<Src>, blocks, SCAN_T, src, wk);
  L.launch(k_border_canon<T, Src>, tiles, 64, src, wk);
  // The relabeling of tiles of 8192 pixels or more runs with 512 threads
  // whatever the other kernels use: it is bound by memory latency and its
  // LDS (not wave slots) limits the workgroups per CU, so wider workgroups
  // keep more waves in flight (measured: faster than 256 and than 1024).
  using TE = Tile<T::TH, T::TW, (T::N >= 8192 && T::NT < 512 ? 512 : T::NT), T::FG8, T::SUP, T::RHT>;
  L.launch(k_tile_emit<TE, Src>, tiles, TE::NT, src, wk);
}

}  // namespace ccl
