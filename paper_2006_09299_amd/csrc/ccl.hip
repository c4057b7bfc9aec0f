// ccl.hip -- C-ABI of libccl.so: argument checks, workspace layout and the
// launch sequence of ccl_pipeline.h on a HIP stream (gfx950).
//
// Variants: the same path compiled for several tile shapes and for the two
// root-reduction schemes (LDS hash per tile group / direct atomics).  The
// batch entry points and the tuner pick one by index; ccl_label uses 0.
#include <hip/hip_runtime.h>

#include <string.h>

#include <mutex>

#include "ccl_pipeline.h"
#include "ccl_fill.h"
#include "../../include/ccl.h"

namespace {

static_assert(sizeof(ccl::Feature) == sizeof(ccl_feature_t), "feature record layout");
static_assert(sizeof(ccl::ImgDesc) <= 256, "the serving footprint counts one 256-byte block per descriptor");

template <int TH, int TW, bool HASH, int NT = 256, bool FG8 = true, int SUP = 4, int RHT = 0>
struct V {
  using T = ccl::Tile<TH, TW, NT, FG8, SUP, RHT>;
  static constexpr bool hash = HASH;
};

// the complementary connectivity pair (4-adjacent foreground, 8-adjacent
// background) in the default variant's shape
using VC4 = V<64, 128, true, 256, false>;
// the default shape with super-tiles of 8 x 8 tiles (variant 9)
using VSUP8 = V<64, 128, true, 256, true, 8>;

// variant index -> (tile rows, tile columns, reduction, workgroup size,
// super-tile side, tiles per root-reduction workgroup)
constexpr int NVARIANTS = 13;

template <class F>
int with_variant(int v, F&& f) {
  switch (v) {
    case 0: return f(V<64, 128, true>{});
    case 1: return f(V<32, 128, false>{});
    case 2: return f(V<16, 128, true>{});
    case 3: return f(V<32, 256, true, 512>{});
    case 4: return f(V<64, 128, true, 512>{});
    case 5: return f(V<32, 128, true>{});
    case 6: return f(V<16, 256, true>{});
    case 7: return f(V<32, 256, true>{});
    // merge schedule: super-tiles of 2 x 2 or 8 x 8 tiles, smaller
    // root-reduction groups
    case 8: return f(V<64, 128, true, 256, true, 2>{});
    case 9: return f(VSUP8{});
    case 10: return f(V<64, 128, true, 512, true, 8>{});
    case 11: return f(V<64, 128, true, 256, true, 4, 16>{});
    case 12: return f(V<32, 128, true, 256, true, 8, 32>{});
    default: return CCL_EINVAL;
  }
}

struct HipLauncher {
  hipStream_t stream;
  hipError_t err = hipSuccess;
  void* const* events = nullptr;  // optional: one event recorded before each kernel
  int k = 0;
  template <class K, class... A>
  void launch(K kernel, int64_t grid, int block, A... args) {
    if (err != hipSuccess) return;
    if (events) err = hipEventRecord(static_cast<hipEvent_t>(events[k++]), stream);
    if (err != hipSuccess || grid <= 0) return;
    hipLaunchKernelGGL(kernel, dim3((unsigned)grid), dim3((unsigned)block), 0, stream, args...);
    err = hipGetLastError();
  }
  void finish() {
    if (events && err == hipSuccess) err = hipEventRecord(static_cast<hipEvent_t>(events[k++]), stream);
  }
};

bool image_args_ok(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out) {
  if (!img || !out || !out->counts || w <= 0 || h <= 0 || pitch < w) return false;
  if ((int64_t)w * h >= INT32_MAX) return false;
  if ((out->features || out->parent || out->color) && out->cap < 1) return false;
  return true;
}

ccl::ImgDesc to_desc(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out) {
  ccl::ImgDesc d;
  memset(&d, 0, sizeof(d));
  d.img = img;
  d.pitch = pitch;
  d.w = w;
  d.h = h;
  d.labels = out->labels;
  d.feat = reinterpret_cast<ccl::Feature*>(out->features);
  d.parent = out->parent;
  d.color = out->color;
  d.cap = out->cap;
  d.counts = out->counts;
  d.flags = 0;
  if ((reinterpret_cast<uintptr_t>(img) & 15) == 0 && (pitch & 15) == 0) d.flags |= ccl::DF_VEC_IN;
  if (out->labels && (reinterpret_cast<uintptr_t>(out->labels) & 15) == 0 && (w & 3) == 0) d.flags |= ccl::DF_VEC_LAB;
  return d;
}

struct Totals {
  int64_t tiles = 0, nodes = 0, cells = 0, blocks = 0, items = 0, supers = 0;
  bool too_big() const { return nodes >= INT32_MAX || tiles >= INT32_MAX || blocks >= INT32_MAX; }
};

// digest of a batch's launch shape: the variant's compile-time shape and the
// totals the descriptors were placed for (FNV-1a over the values)
template <class Vt>
uint32_t batch_check(const Totals& t, int32_t n) {
  using T = typename Vt::T;
  const int64_t v[] = {T::TH, T::TW, T::NT, Vt::hash ? 1 : 0, T::FG8 ? 1 : 0, T::SUP, T::RHT, t.tiles, t.nodes,
                       t.cells, t.blocks, t.items, t.supers, n};
  uint32_t h = 2166136261u;
  for (int64_t x : v)
    for (int b = 0; b < 8; b++) h = (h ^ (uint32_t)((uint64_t)x >> (8 * b) & 0xFF)) * 16777619u;
  return h;
}

// geometry of a batch under variant Vt; fills ds (may be null) with the
// batch's check digest
template <class Vt>
int place_batch(const ccl_image_t* imgs, int32_t n, ccl::ImgDesc* ds, Totals& t) {
  for (int32_t i = 0; i < n; i++) {
    const ccl_image_t& im = imgs[i];
    if (!image_args_ok(im.img, im.w, im.h, im.pitch, &im.out)) return CCL_EINVAL;
    ccl::ImgDesc d = to_desc(im.img, im.w, im.h, im.pitch, &im.out);
    ccl::place_image<typename Vt::T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items, t.supers);
    if (ds) ds[i] = d;
  }
  if (t.too_big()) return CCL_ETOOBIG;
  if (ds) {
    const uint32_t c = batch_check<Vt>(t, n);
    for (int32_t i = 0; i < n; i++) ds[i].check = c;
  }
  return CCL_OK;
}

// Variant of the single-image calls: smaller tiles for smaller images, where
// the chain of phases of one tile is most of the time (p = 0.5 random
// images: 16 x 128 tiles 23 % faster than 64 x 128 at 512^2 and 31 % at
// 1024^2, 32 x 128 tiles 23 % faster at 2048^2; 64 x 128 from 8192^2 up).
// Super-tiles of 8 x 8 tiles once their grid holds 256 workgroups or more:
// k_seam_local then merges 7 / 8 of the seams in LDS instead of 3 / 4
// (16384^2 images 2-7 % faster, random or structured, 12288^2 up to 3 %;
// 8192^2, 128 super-tiles, 3 % slower).
int32_t single_variant(int32_t w, int32_t h) {
  const int64_t px = (int64_t)w * h;
  if (px <= (int64_t)3 << 19) return 2;  // 1.5 Mpixel
  if (px <= (int64_t)6 << 20) return 5;
  using T8 = VSUP8::T;
  const int64_t supers = ((int64_t)w + T8::TW * T8::SUP - 1) / (T8::TW * T8::SUP) *
                         (((int64_t)h + T8::TH * T8::SUP - 1) / (T8::TH * T8::SUP));
  return supers >= 256 ? 9 : 0;
}

int label_one(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
              size_t ws_bytes, void* stream, void* const* events, int32_t variant, bool fg8 = true) {
  if (!image_args_ok(img, w, h, pitch, out) || !ws) return CCL_EINVAL;
  auto pick = [&](auto&& f) -> int { return fg8 ? with_variant(variant, f) : f(VC4{}); };
  return pick([&](auto vt) -> int {
    using Vt = decltype(vt);
    using T = typename Vt::T;
    ccl::ImgDesc d = to_desc(img, w, h, pitch, out);
    Totals t;
    ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items, t.supers);
    if (t.too_big()) return CCL_ETOOBIG;
    ccl::Layout L = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks);
    if (ws_bytes < L.bytes) return CCL_ENOSPC;
    ccl::Work wk = ccl::make_work(L, ws);
    HipLauncher hl{static_cast<hipStream_t>(stream)};
    hl.events = events;
    ccl::OneImage src{d};
    ccl::enqueue<T, Vt::hash>(hl, src, wk, t.tiles, t.items, t.blocks, t.supers);
    hl.finish();
    return hl.err == hipSuccess ? CCL_OK : CCL_EHIP;
  });
}

// workspace of the hole filling: top-level ancestor, filled id and map per
// table entry, block counts
struct FillLayout {
  int64_t nblk;
  size_t off_top, off_fid, off_map, off_bsum, bytes;
};

FillLayout fill_layout(int64_t cap) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  FillLayout L;
  L.nblk = (cap + ccl::fill::FB - 1) / ccl::fill::FB;
  size_t o = 0;
  L.off_top = o;
  o += al(4 * (size_t)cap);
  L.off_fid = o;
  o += al(4 * (size_t)cap);
  L.off_map = o;
  o += al(4 * (size_t)cap);
  L.off_bsum = o;
  o += al(4 * (size_t)L.nblk);
  L.bytes = o;
  return L;
}

// Workspace of ccl_label_noalloc: one array per GPU, a module global of the
// code object (the runtime places it when the library's code is loaded on a
// device; it lives until the process ends).  In host code `scratch` is only
// the host-side handle of the symbol, never a device address: kernels get
// the address hipGetSymbolAddress returns for the current device.
static __device__ __attribute__((used)) __align__(256) unsigned char scratch[CCL_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES];

// address of the current device's scratch (resolved once per device);
// nullptr when the runtime cannot tell
void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" {

int ccl_label_noalloc(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out,
                      void* stream) {
  if (!image_args_ok(img, w, h, pitch, out)) return CCL_EINVAL;
  if (ccl_workspace_bytes(w, h) > CCL_NOALLOC_SCRATCH_BYTES) return CCL_ENOSPC;
  void* ws = scratch_address();
  if (!ws) return CCL_EHIP;
  return label_one(img, w, h, pitch, out, ws, CCL_NOALLOC_SCRATCH_BYTES, stream, nullptr, single_variant(w, h));
}

size_t ccl_fill_workspace_bytes(int64_t cap) {
  if (cap < 1 || cap >= INT32_MAX) return 0;
  return fill_layout(cap).bytes;
}

int ccl_fill_holes(const ccl_outputs_t* in, int32_t w, int32_t h, const ccl_outputs_t* out, int32_t* map, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!in || !out || !ws || !in->parent || !in->counts || !out->counts) return CCL_EINVAL;
  if (in->cap < 1 || in->cap >= INT32_MAX || w <= 0 || h <= 0 || (int64_t)w * h >= INT32_MAX) return CCL_EINVAL;
  if ((out->labels && !in->labels) || (out->features && !in->features)) return CCL_EINVAL;
  if ((out->features || out->parent || out->color) && out->cap < 1) return CCL_EINVAL;
  const FillLayout L = fill_layout(in->cap);
  if (ws_bytes < L.bytes) return CCL_ENOSPC;
  uint8_t* b = static_cast<uint8_t*>(ws);
  ccl::fill::Args a;
  a.labels = in->labels;
  a.feat = reinterpret_cast<const ccl::Feature*>(in->features);
  a.parent = in->parent;
  a.counts = in->counts;
  a.cap = in->cap;
  a.npx = (int64_t)w * h;
  a.olabels = out->labels;
  a.ofeat = reinterpret_cast<ccl::Feature*>(out->features);
  a.oparent = out->parent;
  a.ocolor = out->color;
  a.ocap = out->cap;
  a.ocounts = out->counts;
  a.top = reinterpret_cast<int32_t*>(b + L.off_top);
  a.fid = reinterpret_cast<int32_t*>(b + L.off_fid);
  a.map = map ? map : reinterpret_cast<int32_t*>(b + L.off_map);
  a.bsum = reinterpret_cast<int32_t*>(b + L.off_bsum);
  a.nblk = L.nblk;
  using namespace ccl::fill;
  HipLauncher hl{static_cast<hipStream_t>(stream)};
  hl.launch(k_fill_top, L.nblk, FT, a);
  hl.launch(k_fill_scan, 1, SCAN_WG, a);
  hl.launch(k_fill_ids, L.nblk, FT, a);
  hl.launch(k_fill_merge, (a.cap + FBM - 1) / FBM, FT, a);
  if (out->labels) {
    int64_t blocks = (a.npx / 4 + FT - 1) / FT;
    blocks = blocks < 1 ? 1 : (blocks > 16384 ? 16384 : blocks);
    hl.launch(k_fill_labels, blocks, FT, a);
  }
  return hl.err == hipSuccess ? CCL_OK : CCL_EHIP;
}

int32_t ccl_num_variants(void) { return NVARIANTS; }

int ccl_variant_info(int32_t variant, int32_t* tile_h, int32_t* tile_w, int32_t* hash_reduce, int32_t* threads,
                     int32_t* super_tile, int32_t* reduce_group) {
  return with_variant(variant, [&](auto vt) -> int {
    using Vt = decltype(vt);
    if (tile_h) *tile_h = Vt::T::TH;
    if (tile_w) *tile_w = Vt::T::TW;
    if (hash_reduce) *hash_reduce = Vt::hash ? 1 : 0;
    if (threads) *threads = Vt::T::NT;
    if (super_tile) *super_tile = Vt::T::SUP;
    if (reduce_group) *reduce_group = Vt::hash ? Vt::T::RHT : 1;
    return CCL_OK;
  });
}

size_t ccl_workspace_bytes_v(int32_t w, int32_t h, int32_t variant) {
  if (w <= 0 || h <= 0) return 0;
  size_t bytes = 0;
  with_variant(variant, [&](auto vt) -> int {
    using T = typename decltype(vt)::T;
    ccl::ImgDesc d;
    memset(&d, 0, sizeof(d));
    d.w = w;
    d.h = h;
    Totals t;
    ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items, t.supers);
    bytes = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks).bytes;
    return CCL_OK;
  });
  return bytes;
}

size_t ccl_workspace_bytes(int32_t w, int32_t h) {
  if (w <= 0 || h <= 0) return 0;
  return ccl_workspace_bytes_v(w, h, single_variant(w, h));
}

int32_t ccl_variant_for(int32_t w, int32_t h) { return w > 0 && h > 0 ? single_variant(w, h) : CCL_EINVAL; }

int ccl_label(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
              size_t ws_bytes, void* stream) {
  if (w <= 0 || h <= 0) return CCL_EINVAL;
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, nullptr, single_variant(w, h));
}

int ccl_label_v(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
                size_t ws_bytes, void* stream, int32_t variant) {
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, nullptr, variant);
}

int ccl_label_conn(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
                   size_t ws_bytes, void* stream, int32_t fg_adjacency) {
  if (fg_adjacency != 8 && fg_adjacency != 4) return CCL_EINVAL;
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, nullptr, 0, fg_adjacency == 8);
}

int ccl_label_traced(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
                     size_t ws_bytes, void* stream, void* const* events) {
  if (!events || w <= 0 || h <= 0) return CCL_EINVAL;
  for (int i = 0; i < CCL_TRACE_EVENTS; i++)
    if (!events[i]) return CCL_EINVAL;
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, events, single_variant(w, h));
}

const char* ccl_kernel_name(int k) {
  static const char* names[CCL_TRACE_EVENTS - 1] = {
      "k_tile_export", "k_seam_local", "k_border_merge", "k_reduce_roots", "k_leaders",
      "k_scan_reduce", "k_scan_apply", "k_border_canon", "k_tile_emit"};
  return k >= 0 && k < CCL_TRACE_EVENTS - 1 ? names[k] : nullptr;
}

int ccl_batch_sizes(const ccl_image_t* imgs, int32_t n, int32_t variant, size_t* desc_bytes, size_t* ws_bytes) {
  if (!imgs || n <= 0 || !desc_bytes || !ws_bytes) return CCL_EINVAL;
  return with_variant(variant, [&](auto vt) -> int {
    using Vt = decltype(vt);
    Totals t;
    int rc = place_batch<Vt>(imgs, n, nullptr, t);
    if (rc != CCL_OK) return rc;
    *desc_bytes = sizeof(ccl::ImgDesc) * (size_t)n;
    *ws_bytes = ccl::make_layout<typename Vt::T>(t.tiles, t.nodes, t.cells, t.blocks).bytes;
    return CCL_OK;
  });
}

int ccl_batch_prepare(const ccl_image_t* imgs, int32_t n, int32_t variant, void* host_desc, size_t desc_bytes) {
  if (!imgs || n <= 0 || !host_desc || desc_bytes < sizeof(ccl::ImgDesc) * (size_t)n) return CCL_EINVAL;
  return with_variant(variant, [&](auto vt) -> int {
    Totals t;
    return place_batch<decltype(vt)>(imgs, n, static_cast<ccl::ImgDesc*>(host_desc), t);
  });
}

int ccl_label_batch(const ccl_image_t* imgs, int32_t n, int32_t variant, const void* dev_desc, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!imgs || n <= 0 || !dev_desc || !ws) return CCL_EINVAL;
  return with_variant(variant, [&](auto vt) -> int {
    using Vt = decltype(vt);
    using T = typename Vt::T;
    Totals t;
    int rc = place_batch<Vt>(imgs, n, nullptr, t);
    if (rc != CCL_OK) return rc;
    ccl::Layout L = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks);
    if (ws_bytes < L.bytes) return CCL_ENOSPC;
    ccl::Work wk = ccl::make_work(L, ws);
    HipLauncher hl{static_cast<hipStream_t>(stream)};
    ccl::ManyImages src{static_cast<const ccl::ImgDesc*>(dev_desc), n, batch_check<Vt>(t, n)};
    ccl::enqueue<T, Vt::hash>(hl, src, wk, t.tiles, t.items, t.blocks, t.supers);
    return hl.err == hipSuccess ? CCL_OK : CCL_EHIP;
  });
}

const char* ccl_strerror(int code) {
  switch (code) {
    case CCL_OK: return "ok";
    case CCL_EINVAL: return "invalid argument";
    case CCL_ENOSPC: return "workspace too small";
    case CCL_EHIP: return "HIP launch failed";
    case CCL_ECAPACITY: return "more labels than table capacity";
    case CCL_ETOOBIG: return "too many union-find nodes for one launch";
    default: return "unknown error";
  }
}

void ccl_tile_shape(int32_t* tile_h, int32_t* tile_w) {
  ccl_variant_info(0, tile_h, tile_w, nullptr, nullptr, nullptr, nullptr);
}

}  // extern "C"
