// Drives the serving front end (ccl_server.cpp) on the CPU against the mock
// HIP runtime in mock/ and stand-ins of the batch entry points, over random
// request mixes, pool sizes and configurations, and checks:
//   - every accepted request is reported exactly once, with its own outputs
//     intact until it is released (no block, workspace or descriptor ever
//     overlaps memory that is still live);
//   - admitted requests never exceed max_slots, micro-batches never exceed
//     max_batch, pool use never exceeds the pool;
//   - a request whose first table is too small runs again with exactly
//     n_labels entries, or is reported CCL_ENOSPC when that can never fit;
//   - with one stream and no relaunch, requests finish in submission order;
//   - batches with too many union-find nodes are split;
//   - a micro-batch that a batch entry point refuses (size query, descriptor
//     preparation or launch) reports each of its requests with that error,
//     frees their blocks and the lane's scratch, and the server goes on;
//   - after the last release the pool is empty, and destroy frees every
//     stream, event and pinned buffer.
// Prints "ok" and exits 0, or prints the failed check and exits 1.
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <map>
#include <vector>

#include "../../paper_2006_09299_amd/csrc/ccl_server.cpp"

int (*mock_event_latency)(void) = nullptr;
int mock_live_streams = 0, mock_live_events = 0, mock_live_pinned = 0;

#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      printf("FAILED %s:%d: %s (scenario %d)\n", __FILE__, __LINE__, #c, \
             g_scenario);                                              \
      exit(1);                                                         \
    }                                                                  \
  } while (0)

static int g_scenario = -1;
static uint64_t g_rng = 1;
static uint32_t rnd() {
  g_rng ^= g_rng << 13;
  g_rng ^= g_rng >> 7;
  g_rng ^= g_rng << 17;
  return (uint32_t)(g_rng >> 11);
}
static int rnd(int n) { return (int)(rnd() % (uint32_t)n); }

// ---- stand-ins of the batch entry points -----------------------------------
static int64_t g_px_limit;  // a batch above this many pixels has "too many nodes"
static int g_max_batch;
static int64_t g_label_range;  // true label count of an image: 1 + checksum % min(w*h, range)
static int64_t g_launches_seen;
// path coverage over all scenarios
static int64_t n_sizes_calls, n_toobig, n_launch_total, n_relaunched, n_refused, n_enospc_done;
// refused micro-batches: an image of one of these shapes makes the stand-in
// of that entry point return CCL_EINVAL (only in scenarios that plant them)
static bool g_poison;
enum { POISON_NONE, POISON_SIZES, POISON_PREPARE, POISON_LAUNCH };
static int poison_of(int32_t w, int32_t h) {
  if (!g_poison) return POISON_NONE;
  if (w == 23 && h == 11) return POISON_SIZES;
  if (w == 17 && h == 19) return POISON_PREPARE;
  if (w == 19 && h == 17) return POISON_LAUNCH;
  return POISON_NONE;
}
static int64_t n_poison_sizes, n_poison_prepare, n_poison_launch, n_failed_reports;

static uint32_t checksum(const uint8_t* p, int32_t w, int32_t h, int64_t pitch) {
  uint32_t s = 2166136261u;
  for (int32_t y = 0; y < h; y++)
    for (int32_t x = 0; x < w; x++) s = (s ^ p[y * pitch + x]) * 16777619u;
  return s;
}
static int64_t true_labels(uint32_t cs, int32_t w, int32_t h) {
  int64_t r = std::min<int64_t>((int64_t)w * h, g_label_range);
  return 1 + (int64_t)(cs % (uint64_t)r);
}

extern "C" {
int32_t ccl_num_variants(void) { return 2; }
size_t ccl_workspace_bytes_v(int32_t w, int32_t h, int32_t variant) { return 1000 + (size_t)w * h / 2 + variant; }
int ccl_batch_sizes(const ccl_image_t* imgs, int32_t n, int32_t variant, size_t* db, size_t* wb) {
  CHECK(imgs && n >= 1 && db && wb);
  n_sizes_calls++;
  int64_t px = 0;
  size_t ws = 0;
  for (int i = 0; i < n; i++) {
    CHECK(imgs[i].img && imgs[i].out.counts && imgs[i].pitch == imgs[i].w);
    if (poison_of(imgs[i].w, imgs[i].h) == POISON_SIZES) {
      n_poison_sizes++;
      return CCL_EINVAL;
    }
    px += (int64_t)imgs[i].w * imgs[i].h;
    ws += ccl_workspace_bytes_v(imgs[i].w, imgs[i].h, variant);
  }
  if (px > g_px_limit) {
    n_toobig++;
    return CCL_ETOOBIG;
  }
  *db = 144 * (size_t)n;
  *wb = ws;
  return CCL_OK;
}
int ccl_batch_prepare(const ccl_image_t* imgs, int32_t n, int32_t, void* host_desc, size_t db) {
  CHECK(db >= 144 * (size_t)n);
  for (int i = 0; i < n; i++)
    if (poison_of(imgs[i].w, imgs[i].h) == POISON_PREPARE) {
      n_poison_prepare++;
      return CCL_EINVAL;
    }
  for (int i = 0; i < n; i++) memcpy(static_cast<char*>(host_desc) + 144 * i, &imgs[i], sizeof(void*));
  return CCL_OK;
}
int ccl_label_batch(const ccl_image_t* imgs, int32_t n, int32_t, const void* dev_desc, void* ws, size_t wb,
                    void* stream) {
  CHECK(n >= 1 && n <= g_max_batch && stream);
  for (int i = 0; i < n; i++)
    if (poison_of(imgs[i].w, imgs[i].h) == POISON_LAUNCH) {
      n_poison_launch++;
      return CCL_EINVAL;
    }
  g_launches_seen++;
  n_launch_total++;
  for (int i = 0; i < n; i++) CHECK(memcmp(static_cast<const char*>(dev_desc) + 144 * i, &imgs[i], sizeof(void*)) == 0);
  memset(ws, 0xAB, wb);  // scratch is scribbled over, as the real path does
  for (int i = 0; i < n; i++) {
    const ccl_image_t& im = imgs[i];
    uint32_t cs = checksum(im.img, im.w, im.h, im.pitch);
    int64_t nl = true_labels(cs, im.w, im.h);
    for (int64_t k = 0; k < (int64_t)im.w * im.h; k++) im.out.labels[k] = (int32_t)cs;
    for (int64_t k = 0; k < std::min(nl, im.out.cap); k++) {
      im.out.features[k].S = (int64_t)cs + k;
      im.out.parent[k] = (int32_t)(cs + (uint32_t)k);
      im.out.color[k] = (uint8_t)((cs + k) & 1);
    }
    im.out.counts[0] = nl;
    im.out.counts[1] = (int64_t)(cs % 1000) - 500;
  }
  return CCL_OK;
}
}

// ---- the test -----------------------------------------------------------------
struct HostReq {
  std::vector<uint8_t> img;
  int32_t w, h;
  int64_t pitch;
  uint32_t cs;
  bool accepted = false, reported = false, released = false;
  int hold = 0;  // polls to keep the result before releasing it
  ccl_done_t done{};
};

static void verify_outputs(const HostReq& r) {
  const ccl_done_t& d = r.done;
  if (d.status != CCL_OK) return;
  for (int64_t k = 0; k < (int64_t)r.w * r.h; k++) CHECK(d.out.labels[k] == (int32_t)r.cs);
  for (int64_t k = 0; k < d.n_labels; k++) {
    CHECK(d.out.features[k].S == (int64_t)r.cs + k);
    CHECK(d.out.parent[k] == (int32_t)(r.cs + (uint32_t)k));
    CHECK(d.out.color[k] == (uint8_t)((r.cs + k) & 1));
  }
}

static int latency_small() { return rnd(4); }
static int latency_none() { return 0; }

static void scenario(int s) {
  g_scenario = s;
  g_rng = 0x9E3779B97F4A7C15ull * (uint64_t)(s + 1);
  ccl_server_config_t cfg;
  cfg.streams = 1 + rnd(4);
  cfg.max_batch = 1 + rnd(8);
  cfg.max_slots = 1 + rnd(12);
  cfg.variant = rnd(2);
  bool relaunch = rnd(2);
  cfg.cap_divisor = relaunch ? (1 << 30) : 4;
  g_label_range = relaunch ? 3000 : 1024;
  g_max_batch = cfg.max_batch;
  g_px_limit = 100000 + rnd(100000);
  mock_event_latency = rnd(3) ? latency_small : latency_none;
  int nreq = 30 + rnd(30);
  g_poison = rnd(3) == 0;
  std::vector<HostReq> reqs(nreq);
  for (auto& r : reqs) {
    r.w = 1 + rnd(rnd(2) ? 300 : 40);
    r.h = 1 + rnd(rnd(2) ? 300 : 40);
    if (g_poison && rnd(8) == 0) {
      static const int shapes[3][2] = {{23, 11}, {17, 19}, {19, 17}};
      const int k = rnd(3);
      r.w = shapes[k][0];
      r.h = shapes[k][1];
    }
    r.pitch = r.w + rnd(9);
    r.img.resize((size_t)r.pitch * r.h);
    for (auto& b : r.img) b = (uint8_t)rnd(256);
    r.cs = checksum(r.img.data(), r.w, r.h, r.pitch);
    r.hold = rnd(3) ? 0 : rnd(20);
  }
  // pool: from "a few of the largest requests" down to tight enough that the
  // largest ones are refused and micro-batches must shrink
  size_t pool_bytes = (size_t)(200000 + rnd(4000000));
  std::vector<uint8_t> pool_mem(pool_bytes + 256);
  void* pool = reinterpret_cast<void*>((reinterpret_cast<uintptr_t>(pool_mem.data()) + 255) & ~(uintptr_t)255);
  ccl_server_t* srv = nullptr;
  CHECK(ccl_server_create(pool, pool_bytes, &cfg, &srv) == CCL_OK && srv);

  int next = 0, reported = 0, accepted = 0, poll_count = 0;
  std::vector<int> order;  // report order of accepted requests
  std::vector<ccl_done_t> done(8);
  while (true) {
    // arrivals: up to three per step
    for (int k = rnd(4); k > 0 && next < nreq; k--, next++) {
      HostReq& r = reqs[next];
      size_t fp = 0;
      CHECK(ccl_server_footprint(srv, r.w, r.h, &fp) == CCL_OK);
      int rc = ccl_server_submit(srv, r.img.data(), r.w, r.h, r.pitch, next);
      if (fp > srv->pool.size()) {
        CHECK(rc == CCL_ENOSPC);
        n_refused++;
      } else {
        CHECK(rc == CCL_OK);
        CHECK(ccl_server_submit(srv, r.img.data(), r.w, r.h, r.pitch, next) == CCL_EINVAL);  // duplicate tag
        r.accepted = true;
        accepted++;
      }
    }
    int32_t nd = -1;
    CHECK(ccl_server_poll(srv, done.data(), (int32_t)done.size(), &nd) == CCL_OK);
    CHECK(nd >= 0 && nd <= (int32_t)done.size());
    poll_count++;
    CHECK(poll_count < 200000);  // never stuck
    for (int i = 0; i < nd; i++) {
      const ccl_done_t& d = done[i];
      CHECK(d.tag >= 0 && d.tag < nreq);
      HostReq& r = reqs[d.tag];
      CHECK(r.accepted && !r.reported);
      r.reported = true;
      r.done = d;
      reported++;
      order.push_back((int)d.tag);
      CHECK(d.w == r.w && d.h == r.h && d.out.counts == nullptr);
      if (poison_of(r.w, r.h) != POISON_NONE) CHECK(d.status == CCL_EINVAL);
      if (d.status == CCL_EINVAL) {  // its micro-batch was refused
        CHECK(g_poison && d.out.labels == nullptr && d.launches <= 2);
        n_failed_reports++;
        continue;
      }
      int64_t nl = true_labels(r.cs, r.w, r.h);
      CHECK(d.n_labels == nl && d.euler == (int64_t)(r.cs % 1000) - 500);
      int64_t cap1 = std::min<int64_t>((int64_t)r.w * r.h + 1, std::max<int64_t>(1024, ((int64_t)r.w * r.h + 1) / cfg.cap_divisor));
      if (nl <= cap1) {
        CHECK(d.status == CCL_OK && d.launches == 1 && d.out.cap == cap1);
      } else if (srv->footprint(r.w, r.h, nl) > srv->pool.size()) {
        CHECK(d.status == CCL_ENOSPC && d.launches == 1 && d.out.labels == nullptr);
        n_enospc_done++;
      } else {
        CHECK(d.status == CCL_OK && d.launches == 2 && d.out.cap == nl);
        n_relaunched++;
      }
      verify_outputs(r);
    }
    // releases: results held for a while are checked again before they go
    for (int t = 0; t < nreq; t++) {
      HostReq& r = reqs[t];
      if (!r.reported || r.released) continue;
      if (r.hold-- > 0) continue;
      verify_outputs(r);
      CHECK(ccl_server_release(srv, t) == CCL_OK);
      CHECK(ccl_server_release(srv, t) == CCL_EINVAL);
      r.released = true;
    }
    ccl_server_stats_t st;
    CHECK(ccl_server_stats(srv, &st) == CCL_OK);
    CHECK(st.live <= cfg.max_slots && st.pool_used <= st.pool_bytes && st.in_flight <= cfg.streams);
    if (next == nreq && reported == accepted) {
      bool all = true;
      for (auto& r : reqs) all &= !r.reported || r.released;
      if (all) {
        CHECK(st.queued == 0 && st.in_flight == 0 && st.live == 0 && st.pool_used == 0 && st.ready == 0);
        CHECK(st.completed == accepted && st.launches == g_launches_seen);
        CHECK(st.in_flight == 0);
        break;
      }
    }
  }
  if (cfg.streams == 1 && !relaunch && !g_poison) CHECK(std::is_sorted(order.begin(), order.end()));
  CHECK(ccl_server_destroy(srv) == CCL_OK);
  CHECK(mock_live_streams == 0 && mock_live_events == 0 && mock_live_pinned == 0);
}

int main(int argc, char** argv) {
  int n = argc > 1 ? atoi(argv[1]) : 200;
  for (int s = 0; s < n; s++) {
    g_launches_seen = 0;
    scenario(s);
  }
  // retries: size queries that did not end in a launch (too many nodes, or
  // scratch that did not fit and made the micro-batch shrink)
  printf("ok %d scenarios: launches %lld retries %lld toobig %lld relaunched %lld refused %lld enospc_done %lld "
         "failed_sizes %lld failed_prepare %lld failed_launch %lld failed_reports %lld\n", n,
         (long long)n_launch_total, (long long)(n_sizes_calls - n_launch_total), (long long)n_toobig,
         (long long)n_relaunched, (long long)n_refused, (long long)n_enospc_done, (long long)n_poison_sizes,
         (long long)n_poison_prepare, (long long)n_poison_launch, (long long)n_failed_reports);
  return 0;
}
