// ccl.hip -- C-ABI of libccl.so: argument checks, workspace layout and the
// launch sequence of ccl_pipeline.h on a HIP stream (gfx950).
#include <hip/hip_runtime.h>

#include <string.h>

#include "ccl_pipeline.h"
#include "../../include/ccl.h"

namespace {

using T = ccl::Tile<32, 128>;

static_assert(sizeof(ccl::Feature) == sizeof(ccl_feature_t), "feature record layout");

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
  if ((reinterpret_cast<uintptr_t>(out->labels) & 15) == 0 && (w & 3) == 0) d.flags |= ccl::DF_VEC_LAB;
  return d;
}

struct Totals {
  int64_t tiles = 0, nodes = 0, cells = 0, blocks = 0, items = 0;
};

}  // namespace

extern "C" {

size_t ccl_workspace_bytes(int32_t w, int32_t h) {
  if (w <= 0 || h <= 0) return 0;
  ccl::ImgDesc d;
  memset(&d, 0, sizeof(d));
  d.w = w;
  d.h = h;
  Totals t;
  ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items);
  return ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks).bytes;
}

static int label_one(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
                     size_t ws_bytes, void* stream, void* const* events) {
  if (!image_args_ok(img, w, h, pitch, out) || !ws) return CCL_EINVAL;
  ccl::ImgDesc d = to_desc(img, w, h, pitch, out);
  Totals t;
  ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items);
  if (t.nodes >= INT32_MAX) return CCL_ETOOBIG;
  ccl::Layout L = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks);
  if (ws_bytes < L.bytes) return CCL_ENOSPC;
  ccl::Work wk = ccl::make_work(L, ws);
  HipLauncher hl{static_cast<hipStream_t>(stream)};
  hl.events = events;
  ccl::OneImage src{d};
  ccl::enqueue<T>(hl, src, wk, t.tiles, t.items, t.blocks, 1);
  hl.finish();
  return hl.err == hipSuccess ? CCL_OK : CCL_EHIP;
}

int ccl_label(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
              size_t ws_bytes, void* stream) {
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, nullptr);
}

int ccl_label_traced(const uint8_t* img, int32_t w, int32_t h, int64_t pitch, const ccl_outputs_t* out, void* ws,
                     size_t ws_bytes, void* stream, void* const* events) {
  if (!events) return CCL_EINVAL;
  for (int i = 0; i < CCL_TRACE_EVENTS; i++)
    if (!events[i]) return CCL_EINVAL;
  return label_one(img, w, h, pitch, out, ws, ws_bytes, stream, events);
}

const char* ccl_kernel_name(int k) {
  static const char* names[CCL_TRACE_EVENTS - 1] = {
      "k_tile_export", "k_border_merge", "k_flatten", "k_reduce_roots", "k_leaders",
      "k_scan_reduce", "k_scan_blocks", "k_scan_apply", "k_emit_border", "k_tile_emit"};
  return k >= 0 && k < CCL_TRACE_EVENTS - 1 ? names[k] : nullptr;
}

int ccl_batch_sizes(const ccl_image_t* imgs, int32_t n, size_t* desc_bytes, size_t* ws_bytes) {
  if (!imgs || n <= 0 || !desc_bytes || !ws_bytes) return CCL_EINVAL;
  Totals t;
  for (int32_t i = 0; i < n; i++) {
    const ccl_image_t& im = imgs[i];
    if (!image_args_ok(im.img, im.w, im.h, im.pitch, &im.out)) return CCL_EINVAL;
    ccl::ImgDesc d = to_desc(im.img, im.w, im.h, im.pitch, &im.out);
    ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items);
  }
  if (t.nodes >= INT32_MAX || t.tiles >= INT32_MAX || t.blocks >= INT32_MAX) return CCL_ETOOBIG;
  *desc_bytes = sizeof(ccl::ImgDesc) * (size_t)n;
  *ws_bytes = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks).bytes;
  return CCL_OK;
}

int ccl_batch_prepare(const ccl_image_t* imgs, int32_t n, void* host_desc, size_t desc_bytes) {
  if (!imgs || n <= 0 || !host_desc || desc_bytes < sizeof(ccl::ImgDesc) * (size_t)n) return CCL_EINVAL;
  ccl::ImgDesc* ds = static_cast<ccl::ImgDesc*>(host_desc);
  Totals t;
  for (int32_t i = 0; i < n; i++) {
    const ccl_image_t& im = imgs[i];
    if (!image_args_ok(im.img, im.w, im.h, im.pitch, &im.out)) return CCL_EINVAL;
    ds[i] = to_desc(im.img, im.w, im.h, im.pitch, &im.out);
    ccl::place_image<T>(ds[i], t.tiles, t.nodes, t.cells, t.blocks, t.items);
  }
  if (t.nodes >= INT32_MAX || t.tiles >= INT32_MAX || t.blocks >= INT32_MAX) return CCL_ETOOBIG;
  return CCL_OK;
}

int ccl_label_batch(const ccl_image_t* imgs, int32_t n, const void* dev_desc, void* ws, size_t ws_bytes,
                    void* stream) {
  if (!imgs || n <= 0 || !dev_desc || !ws) return CCL_EINVAL;
  Totals t;
  for (int32_t i = 0; i < n; i++) {
    const ccl_image_t& im = imgs[i];
    if (!image_args_ok(im.img, im.w, im.h, im.pitch, &im.out)) return CCL_EINVAL;
    ccl::ImgDesc d = to_desc(im.img, im.w, im.h, im.pitch, &im.out);
    ccl::place_image<T>(d, t.tiles, t.nodes, t.cells, t.blocks, t.items);
  }
  if (t.nodes >= INT32_MAX || t.tiles >= INT32_MAX || t.blocks >= INT32_MAX) return CCL_ETOOBIG;
  ccl::Layout L = ccl::make_layout<T>(t.tiles, t.nodes, t.cells, t.blocks);
  if (ws_bytes < L.bytes) return CCL_ENOSPC;
  ccl::Work wk = ccl::make_work(L, ws);
  HipLauncher hl{static_cast<hipStream_t>(stream)};
  ccl::ManyImages src{static_cast<const ccl::ImgDesc*>(dev_desc), n};
  ccl::enqueue<T>(hl, src, wk, t.tiles, t.items, t.blocks, n);
  return hl.err == hipSuccess ? CCL_OK : CCL_EHIP;
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
  if (tile_h) *tile_h = T::TH;
  if (tile_w) *tile_w = T::TW;
}

}  // extern "C"
