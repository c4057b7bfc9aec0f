// ccl_server.cpp -- serving front end of libccl.so: continuous batching over
// ccl_label_batch, admission by device footprint, micro-batches on several
// HIP streams.  Host code only; every step of the labeling runs in the
// kernels behind ccl_label_batch.
#include <hip/hip_runtime_api.h>

#include <stdint.h>
#include <string.h>

#include <deque>
#include <new>
#include <unordered_map>
#include <vector>

#include "ccl_pool.h"
#include "../../include/ccl.h"

namespace ccl_serving {

enum Blk { B_IN, B_LAB, B_FEAT, B_PAR, B_COL, NBLK };
enum State { QUEUED, IN_FLIGHT, DONE };

constexpr int MAX_STREAMS = 16;
constexpr size_t COUNTS_BYTES = 2 * sizeof(int64_t);

struct Req {
  const uint8_t* img = nullptr;
  int32_t w = 0, h = 0;
  int64_t pitch = 0;
  int64_t cap = 0;
  size_t off[NBLK] = {}, len[NBLK] = {};
  bool has_blocks = false;
  State st = QUEUED;
  int32_t status = CCL_OK;
  int32_t launches = 0;
  int64_t n_labels = 0, euler = 0;
};

// grow-only pinned host buffer; regrown only while no copy from or to it runs
struct Pinned {
  void* p = nullptr;
  size_t n = 0;
  bool ensure(size_t bytes) {
    if (bytes <= n) return true;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      return false;
    }
    n = bytes;
    return true;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    n = 0;
  }
};

// one stream and the micro-batch it carries
struct Lane {
  hipStream_t stream = nullptr;
  hipEvent_t finished = nullptr;
  bool busy = false;
  std::vector<int64_t> tags;
  std::vector<ccl_image_t> imgs;
  size_t ws_off = 0, ws_len = 0, desc_off = 0, desc_len = 0, cnt_off = 0, cnt_len = 0;
  Pinned desc, counts;
};

}  // namespace ccl_serving

using namespace ccl_serving;

struct ccl_server {
  uint8_t* base = nullptr;
  ccl::Pool pool;
  ccl_server_config_t cfg{};
  Lane lanes[MAX_STREAMS];
  int next_lane = 0;
  std::unordered_map<int64_t, Req> reqs;
  std::deque<int64_t> queue;  // submitted, not admitted; relaunches go to the front
  std::deque<int64_t> ready;  // finished, not yet returned by poll
  int64_t live = 0;
  int64_t in_flight = 0;
  int64_t admitted = 0, completed = 0, launches = 0, relaunched = 0;
  int broken = CCL_OK;

  int64_t first_cap(int32_t w, int32_t h) const {
    int64_t full = (int64_t)w * h + 1, c = full / cfg.cap_divisor;
    if (c < 1024) c = 1024;
    return c < full ? c : full;
  }

  void block_sizes(const Req& r, size_t* len) const {
    size_t px = (size_t)r.w * (size_t)r.h;
    len[B_IN] = px;
    len[B_LAB] = 4 * px;
    len[B_FEAT] = sizeof(ccl_feature_t) * (size_t)r.cap;
    len[B_PAR] = 4 * (size_t)r.cap;
    len[B_COL] = (size_t)r.cap;
  }

  size_t footprint(int32_t w, int32_t h, int64_t cap) const {
    Req r;
    r.w = w;
    r.h = h;
    r.cap = cap;
    size_t len[NBLK], total = 0;
    block_sizes(r, len);
    for (int b = 0; b < NBLK; b++) total += ccl::Pool::round(len[b]);
    // one descriptor is at most 256 bytes; the workspace of a batch of one
    // image is that image's workspace
    total += ccl::Pool::ALIGN + ccl::Pool::round(ccl_workspace_bytes_v(w, h, cfg.variant)) +
             ccl::Pool::round(COUNTS_BYTES);
    return total;
  }

  bool take_blocks(Req& r) {
    size_t len[NBLK];
    block_sizes(r, len);
    for (int b = 0; b < NBLK; b++) {
      size_t off = pool.alloc(len[b]);
      if (off == ccl::Pool::NONE) {
        for (int c = 0; c < b; c++) pool.release(r.off[c], r.len[c]);
        return false;
      }
      r.off[b] = off;
      r.len[b] = len[b];
    }
    r.has_blocks = true;
    live++;
    return true;
  }

  void drop_blocks(Req& r) {
    if (!r.has_blocks) return;
    for (int b = 0; b < NBLK; b++) pool.release(r.off[b], r.len[b]);
    r.has_blocks = false;
    live--;
  }

  int fail(hipError_t e) {
    if (e != hipSuccess && broken == CCL_OK) broken = CCL_EHIP;
    return broken;
  }

  ccl_image_t image_of(const Req& r, int64_t* counts_dev) const {
    ccl_image_t im;
    memset(&im, 0, sizeof(im));
    im.img = base + r.off[B_IN];
    im.w = r.w;
    im.h = r.h;
    im.pitch = r.w;
    im.out.labels = reinterpret_cast<int32_t*>(base + r.off[B_LAB]);
    im.out.features = reinterpret_cast<ccl_feature_t*>(base + r.off[B_FEAT]);
    im.out.parent = reinterpret_cast<int32_t*>(base + r.off[B_PAR]);
    im.out.color = base + r.off[B_COL];
    im.out.cap = r.cap;
    im.out.counts = counts_dev;
    return im;
  }

  // collect every finished micro-batch
  int collect() {
    for (int l = 0; l < cfg.streams; l++) {
      Lane& L = lanes[l];
      if (!L.busy) continue;
      hipError_t e = hipEventQuery(L.finished);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return fail(e);
      const int64_t* c = static_cast<const int64_t*>(L.counts.p);
      std::vector<int64_t> again;
      for (size_t i = 0; i < L.tags.size(); i++) {
        Req& r = reqs[L.tags[i]];
        int64_t n = c[2 * i], eu = c[2 * i + 1];
        r.n_labels = n;
        r.euler = eu;
        if (n > r.cap) {
          // the tables were too small: run again with exactly n entries, if
          // that can ever fit the pool
          drop_blocks(r);
          if (footprint(r.w, r.h, n) > pool.size()) {
            r.status = CCL_ENOSPC;
            r.st = DONE;
            ready.push_back(L.tags[i]);
            completed++;
          } else {
            r.cap = n;
            r.st = QUEUED;
            again.push_back(L.tags[i]);
            relaunched++;
          }
        } else {
          r.st = DONE;
          ready.push_back(L.tags[i]);
          completed++;
        }
      }
      for (size_t i = again.size(); i-- > 0;) queue.push_front(again[i]);
      pool.release(L.ws_off, L.ws_len);
      pool.release(L.desc_off, L.desc_len);
      pool.release(L.cnt_off, L.cnt_len);
      L.tags.clear();
      L.busy = false;
      in_flight--;
    }
    return CCL_OK;
  }

  // a micro-batch that cannot be launched: each of its requests is reported
  // with the error (its blocks go back to the pool), and so is the lane's
  // scratch when it was taken
  void abort_batch(Lane& L, int rc, bool scratch) {
    if (scratch) {
      pool.release(L.ws_off, L.ws_len);
      pool.release(L.desc_off, L.desc_len);
      pool.release(L.cnt_off, L.cnt_len);
    }
    for (int64_t tag : L.tags) {
      Req& r = reqs[tag];
      drop_blocks(r);
      r.status = rc;
      r.st = DONE;
      ready.push_back(tag);
      completed++;
    }
    L.tags.clear();
  }

  // admit queue heads into one micro-batch and launch it on lane L
  int launch(Lane& L) {
    std::vector<int64_t>& batch = L.tags;
    batch.clear();
    while (!queue.empty() && (int64_t)batch.size() < cfg.max_batch && live < cfg.max_slots) {
      Req& r = reqs[queue.front()];
      if (!take_blocks(r)) break;
      batch.push_back(queue.front());
      queue.pop_front();
    }
    if (batch.empty()) return CCL_OK;
    size_t db = 0, wb = 0;
    for (;;) {
      size_t n = batch.size();
      L.imgs.resize(n);
      // the counts pointers are placed once the counts block exists; the
      // sizes do not depend on them, but the argument check wants them set
      for (size_t i = 0; i < n; i++) L.imgs[i] = image_of(reqs[batch[i]], reinterpret_cast<int64_t*>(base));
      int rc = ccl_batch_sizes(L.imgs.data(), (int32_t)n, cfg.variant, &db, &wb);
      if (rc != CCL_OK && !(rc == CCL_ETOOBIG && n > 1)) {
        abort_batch(L, rc, false);
        return CCL_OK;
      }
      if (rc == CCL_OK) {
        L.ws_off = pool.alloc(wb);
        L.desc_off = L.ws_off == ccl::Pool::NONE ? ccl::Pool::NONE : pool.alloc(db);
        L.cnt_off = L.desc_off == ccl::Pool::NONE ? ccl::Pool::NONE : pool.alloc(COUNTS_BYTES * n);
        if (L.cnt_off != ccl::Pool::NONE) break;
        if (L.desc_off != ccl::Pool::NONE) pool.release(L.desc_off, db);
        if (L.ws_off != ccl::Pool::NONE) pool.release(L.ws_off, wb);
      }
      // the micro-batch's scratch does not fit (or it has too many union-find
      // nodes for one launch): hand the last request back to the queue head
      // and try a smaller one
      Req& last = reqs[batch.back()];
      drop_blocks(last);
      queue.push_front(batch.back());
      batch.pop_back();
      if (batch.empty()) return CCL_OK;  // wait for memory to come back
    }
    size_t n = batch.size();
    L.ws_len = wb;
    L.desc_len = db;
    L.cnt_len = COUNTS_BYTES * n;
    int64_t* cnt = reinterpret_cast<int64_t*>(base + L.cnt_off);
    for (size_t i = 0; i < n; i++) L.imgs[i].out.counts = cnt + 2 * i;
    if (!L.desc.ensure(db) || !L.counts.ensure(L.cnt_len)) return fail(hipErrorOutOfMemory);
    int rc = ccl_batch_prepare(L.imgs.data(), (int32_t)n, cfg.variant, L.desc.p, db);
    if (rc != CCL_OK) {
      abort_batch(L, rc, true);
      return CCL_OK;
    }
    for (size_t i = 0; i < n; i++) {
      Req& r = reqs[batch[i]];
      hipError_t e = r.pitch == r.w
                         ? hipMemcpyAsync(base + r.off[B_IN], r.img, (size_t)r.w * r.h, hipMemcpyHostToDevice, L.stream)
                         : hipMemcpy2DAsync(base + r.off[B_IN], (size_t)r.w, r.img, (size_t)r.pitch, (size_t)r.w,
                                            (size_t)r.h, hipMemcpyHostToDevice, L.stream);
      if (e != hipSuccess) return fail(e);
      r.st = IN_FLIGHT;
      r.launches++;
    }
    hipError_t e = hipMemcpyAsync(base + L.desc_off, L.desc.p, db, hipMemcpyHostToDevice, L.stream);
    if (e != hipSuccess) return fail(e);
    rc = ccl_label_batch(L.imgs.data(), (int32_t)n, cfg.variant, base + L.desc_off, base + L.ws_off, wb, L.stream);
    if (rc == CCL_EHIP) return fail(hipErrorLaunchFailure);
    if (rc != CCL_OK) {
      // the uploads are already enqueued: the host images stay in use until
      // they are done
      e = hipStreamSynchronize(L.stream);
      if (e != hipSuccess) return fail(e);
      abort_batch(L, rc, true);
      return CCL_OK;
    }
    e = hipMemcpyAsync(L.counts.p, cnt, L.cnt_len, hipMemcpyDeviceToHost, L.stream);
    if (e == hipSuccess) e = hipEventRecord(L.finished, L.stream);
    if (e != hipSuccess) return fail(e);
    L.busy = true;
    in_flight++;
    launches++;
    admitted += (int64_t)n;
    return CCL_OK;
  }
};

extern "C" {

int ccl_server_create(void* pool, size_t pool_bytes, const ccl_server_config_t* cfg, ccl_server_t** srv) {
  if (!srv) return CCL_EINVAL;
  *srv = nullptr;
  ccl_server_config_t c = cfg ? *cfg : ccl_server_config_t{256, 4, 64, 0, 4};
  if (!pool || (reinterpret_cast<uintptr_t>(pool) & (ccl::Pool::ALIGN - 1)) || pool_bytes < ccl::Pool::ALIGN)
    return CCL_EINVAL;
  if (c.max_slots < 1 || c.streams < 1 || c.streams > MAX_STREAMS || c.max_batch < 1 || c.cap_divisor < 1 ||
      c.variant < 0 || c.variant >= ccl_num_variants())
    return CCL_EINVAL;
  ccl_server* s = new (std::nothrow) ccl_server;
  if (!s) return CCL_EINVAL;
  s->base = static_cast<uint8_t*>(pool);
  s->pool.reset(pool_bytes);
  s->cfg = c;
  for (int l = 0; l < c.streams; l++) {
    hipError_t e = hipStreamCreateWithFlags(&s->lanes[l].stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->lanes[l].finished, hipEventDisableTiming);
    if (e != hipSuccess) {
      s->cfg.streams = l + 1;
      ccl_server_destroy(s);
      return CCL_EHIP;
    }
  }
  *srv = s;
  return CCL_OK;
}

int ccl_server_footprint(const ccl_server_t* srv, int32_t w, int32_t h, size_t* bytes) {
  if (!srv || !bytes || w <= 0 || h <= 0 || (int64_t)w * h >= INT32_MAX) return CCL_EINVAL;
  *bytes = srv->footprint(w, h, srv->first_cap(w, h));
  return CCL_OK;
}

int ccl_server_submit(ccl_server_t* srv, const uint8_t* img, int32_t w, int32_t h, int64_t pitch, int64_t tag) {
  if (!srv) return CCL_EINVAL;
  if (srv->broken) return srv->broken;
  if (!img || w <= 0 || h <= 0 || pitch < w || (int64_t)w * h >= INT32_MAX) return CCL_EINVAL;
  if (srv->reqs.count(tag)) return CCL_EINVAL;
  int64_t cap = srv->first_cap(w, h);
  if (srv->footprint(w, h, cap) > srv->pool.size()) return CCL_ENOSPC;
  Req& r = srv->reqs[tag];
  r.img = img;
  r.w = w;
  r.h = h;
  r.pitch = pitch;
  r.cap = cap;
  srv->queue.push_back(tag);
  return CCL_OK;
}

int ccl_server_poll(ccl_server_t* srv, ccl_done_t* done, int32_t max_done, int32_t* n_done) {
  if (!srv || !n_done || max_done < 0 || (max_done > 0 && !done)) return CCL_EINVAL;
  *n_done = 0;
  if (srv->broken) return srv->broken;
  int rc = srv->collect();
  if (rc != CCL_OK) return rc;
  // one micro-batch per idle stream, round robin over the streams
  for (int k = 0; k < srv->cfg.streams && !srv->queue.empty(); k++) {
    Lane& L = srv->lanes[srv->next_lane];
    if (L.busy) {
      srv->next_lane = (srv->next_lane + 1) % srv->cfg.streams;
      continue;
    }
    rc = srv->launch(L);
    if (rc != CCL_OK) return rc;
    if (!L.busy) break;  // nothing could be admitted
    srv->next_lane = (srv->next_lane + 1) % srv->cfg.streams;
  }
  int32_t k = 0;
  while (k < max_done && !srv->ready.empty()) {
    int64_t tag = srv->ready.front();
    srv->ready.pop_front();
    const Req& r = srv->reqs[tag];
    ccl_done_t& d = done[k++];
    memset(&d, 0, sizeof(d));
    d.tag = tag;
    d.status = r.status;
    d.w = r.w;
    d.h = r.h;
    d.launches = r.launches;
    d.n_labels = r.n_labels;
    d.euler = r.euler;
    if (r.status == CCL_OK) d.out = srv->image_of(r, nullptr).out;
  }
  *n_done = k;
  return CCL_OK;
}

int ccl_server_release(ccl_server_t* srv, int64_t tag) {
  if (!srv) return CCL_EINVAL;
  auto it = srv->reqs.find(tag);
  if (it == srv->reqs.end() || it->second.st != DONE) return CCL_EINVAL;
  for (auto q = srv->ready.begin(); q != srv->ready.end(); ++q)
    if (*q == tag) {
      srv->ready.erase(q);
      break;
    }
  srv->drop_blocks(it->second);
  srv->reqs.erase(it);
  return CCL_OK;
}

int ccl_server_stats(const ccl_server_t* srv, ccl_server_stats_t* st) {
  if (!srv || !st) return CCL_EINVAL;
  st->queued = (int64_t)srv->queue.size();
  st->live = srv->live;
  st->in_flight = srv->in_flight;
  st->ready = (int64_t)srv->ready.size();
  st->pool_used = (int64_t)srv->pool.used();
  st->pool_bytes = (int64_t)srv->pool.size();
  st->admitted = srv->admitted;
  st->completed = srv->completed;
  st->launches = srv->launches;
  st->relaunched = srv->relaunched;
  return srv->broken;
}

int ccl_server_destroy(ccl_server_t* srv) {
  if (!srv) return CCL_EINVAL;
  int rc = CCL_OK;
  for (int l = 0; l < srv->cfg.streams; l++) {
    Lane& L = srv->lanes[l];
    if (L.stream && hipStreamSynchronize(L.stream) != hipSuccess) rc = CCL_EHIP;
    if (L.finished) (void)hipEventDestroy(L.finished);
    if (L.stream) (void)hipStreamDestroy(L.stream);
    L.desc.release();
    L.counts.release();
  }
  delete srv;
  return rc;
}

}  // extern "C"
