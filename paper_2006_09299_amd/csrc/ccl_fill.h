// ccl_fill.h -- hole filling on a finished labeling (gfx950).
//
// The transitive closure of the paper has an optional step (Sec. 3.2,
// Algorithm 3; Fig. 2, "hole filled"): a component whose surrounding is not
// the exterior is merged into that surrounding, and since the closure runs
// forward, nested levels cascade into the top-level foreground component.
// With the inclusion tree at hand (parent table of the labeling) that is:
// the filled component of c is its top-level ancestor t (parent[t] = exterior),
// the filled image's components are the exterior and the top-level foreground
// components, each with everything nested inside it.
//
// Filled ids keep the canonical rule (exterior 0, others by the raster rank
// of their first pixel): a top-level component's first pixel is also the
// first pixel of its filled region (what it encloses lies below or right of
// it), so the filled id of t is 1 + the number of top-level ids below t.
// Features: S, Sx, Sy of the nested components are added; the bounding box is
// the top-level component's own (an enclosed pixel lies between pixels of its
// surrounding in its row and in its column).
//
// Kernels, one launch each, in this order:
//   k_fill_top    : top-level ancestor of every id (walk up the parent table,
//                   whose entries strictly decrease); top-level ids per block
//   k_fill_scan   : one workgroup: exclusive scan of the block counts; the
//                   filled counts and the exterior's table entries
//   k_fill_ids    : filled id of every top-level id, its table entries
//   k_fill_merge  : filled id of every id (map); S, Sx, Sy of nested ids
//                   added into their filled component
//   k_fill_labels : filled label image = map[label] (optional)
// The number of labels is read on the device (counts[0] of the labeling), so
// the sequence needs no host synchronisation; grids cover the table capacity.
#pragma once

#include <stdint.h>

namespace ccl {
namespace fill {

constexpr int FT = 256;       // threads per workgroup
constexpr int FK = 4;         // ids per thread
constexpr int FB = FT * FK;   // ids per block
constexpr int SCAN_WG = 1024; // threads of the block-count scan

struct Args {
  // the labeling (device)
  const int32_t* labels;   // [npx] or null
  const Feature* feat;     // [cap] or null
  const int32_t* parent;   // [cap]
  const int64_t* counts;   // [2]
  int64_t cap;
  int64_t npx;
  // the filled labeling (device)
  int32_t* olabels;        // [npx] or null
  Feature* ofeat;          // [ocap] or null
  int32_t* oparent;        // [ocap] or null
  uint8_t* ocolor;         // [ocap] or null
  int64_t ocap;
  int64_t* ocounts;        // [2]
  // scratch (device)
  int32_t* map;            // [cap]: filled id of every id
  int32_t* top;            // [cap]: top-level ancestor
  int32_t* fid;            // [cap]: filled id, at top-level ids
  int32_t* bsum;           // [nblk]: top-level ids per block, then block offsets
  int64_t nblk;
};

// the labeling is usable: 1 <= n <= cap (a truncated labeling has n > cap)
__device__ inline int64_t fill_n(const Args& a) {
  const int64_t n = a.counts[0];
  return n >= 1 && n <= a.cap ? n : 0;
}

__device__ inline bool is_top(const Args& a, int64_t c) { return c > 0 && a.parent[c] == 0; }

// workgroup-wide exclusive sum of v over FT threads (total in *tot)
__device__ inline uint32_t fill_block_scan(uint32_t v, uint32_t* tmp, uint32_t* tot) {
  const int t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (int d = 1; d < FT; d <<= 1) {
    uint32_t add = t >= d ? tmp[t - d] : 0u;
    __syncthreads();
    tmp[t] += add;
    __syncthreads();
  }
  *tot = tmp[FT - 1];
  const uint32_t ex = tmp[t] - v;
  __syncthreads();
  return ex;
}

__global__ void __launch_bounds__(FT) k_fill_top(Args a) {
  __shared__ uint32_t tmp[FT];
  const int64_t n = fill_n(a);
  const int64_t c0 = (int64_t)blockIdx.x * FB + (int64_t)threadIdx.x * FK;
  uint32_t cnt = 0;
  for (int k = 0; k < FK; k++) {
    const int64_t c = c0 + k;
    if (c >= n) break;
    // walk up; parent entries strictly decrease down to the exterior, so
    // the walk ends (an entry that does not decrease stops it)
    int32_t t = (int32_t)c;
    if (c > 0) {
      int32_t p = a.parent[t];
      while (p > 0 && p < t) {
        t = p;
        p = a.parent[t];
      }
    }
    a.top[c] = t;
    cnt += is_top(a, c) ? 1u : 0u;
  }
  uint32_t tot;
  (void)fill_block_scan(cnt, tmp, &tot);
  if (threadIdx.x == 0 && (int64_t)blockIdx.x < a.nblk) a.bsum[blockIdx.x] = (int32_t)tot;
}

__global__ void __launch_bounds__(SCAN_WG) k_fill_scan(Args a) {
  __shared__ uint32_t tmp[SCAN_WG];
  const int t = threadIdx.x;
  const int64_t n = fill_n(a);
  const int64_t nb = n ? (n + FB - 1) / FB : 0;
  uint32_t carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_WG) {
    const int64_t b = base + t;
    const uint32_t v = b < nb ? (uint32_t)a.bsum[b] : 0u;
    tmp[t] = v;
    __syncthreads();
    for (int d = 1; d < SCAN_WG; d <<= 1) {
      uint32_t add = t >= d ? tmp[t - d] : 0u;
      __syncthreads();
      tmp[t] += add;
      __syncthreads();
    }
    if (b < nb) a.bsum[b] = (int32_t)(carry + tmp[t] - v);
    carry += tmp[SCAN_WG - 1];
    __syncthreads();
  }
  if (t == 0) {
    if (!n) {  // the labeling's tables were truncated: nothing is filled
      a.ocounts[0] = -1;
      a.ocounts[1] = 0;
      return;
    }
    a.ocounts[0] = 1 + (int64_t)carry;  // the exterior and the top-level components
    a.ocounts[1] = (int64_t)carry;      // no holes are left
    if (a.ocap >= 1) {
      if (a.ofeat && a.feat) a.ofeat[0] = a.feat[0];  // the exterior does not change
      if (a.oparent) a.oparent[0] = -1;
      if (a.ocolor) a.ocolor[0] = 0;
    }
  }
}

__global__ void __launch_bounds__(FT) k_fill_ids(Args a) {
  __shared__ uint32_t tmp[FT];
  const int64_t n = fill_n(a);
  const int64_t c0 = (int64_t)blockIdx.x * FB + (int64_t)threadIdx.x * FK;
  uint32_t cnt = 0;
  for (int k = 0; k < FK; k++) {
    const int64_t c = c0 + k;
    if (c < n && is_top(a, c)) cnt++;
  }
  uint32_t tot;
  uint32_t f = fill_block_scan(cnt, tmp, &tot);
  if (!n || (int64_t)blockIdx.x >= a.nblk) return;
  f += 1u + (uint32_t)a.bsum[blockIdx.x];
  for (int k = 0; k < FK; k++) {
    const int64_t c = c0 + k;
    if (c >= n || !is_top(a, c)) continue;
    a.fid[c] = (int32_t)f;
    if ((int64_t)f < a.ocap) {
      if (a.ofeat && a.feat) a.ofeat[f] = a.feat[c];
      if (a.oparent) a.oparent[f] = 0;
      if (a.ocolor) a.ocolor[f] = 1;
    }
    f++;
  }
}

__device__ inline unsigned long long fill_wave_sum(unsigned long long v) {
  for (int o = 32; o; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline void fill_add(Feature* o, unsigned long long s0, unsigned long long s1, unsigned long long s2) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&o->S), s0);
  atomicAdd(reinterpret_cast<unsigned long long*>(&o->Sx), s1);
  atomicAdd(reinterpret_cast<unsigned long long*>(&o->Sy), s2);
}

// One id per lane and step (a wave covers 64 consecutive ids per step), FKM
// steps per thread.  A percolating top-level component can hold millions of
// nested ids, all adding into the same three counters, whose atomics are
// served one after another: the workgroup takes the target of its first
// contributing id as a candidate, sums every contribution to it (in each
// lane, then over the wave, then in LDS) and adds once per workgroup, so the
// more ids a workgroup covers the fewer such atomics (16 ids per thread:
// -60 % on the 8192^2 sweep against 4); within a wave, contributions to the
// target of the wave's first other lane are summed too; the rest add
// directly.
constexpr int FKM = 16;          // ids per thread of k_fill_merge
constexpr int FBM = FT * FKM;    // ids per workgroup of k_fill_merge
__global__ void __launch_bounds__(FT) k_fill_merge(Args a) {
  __shared__ int32_t wcand[FT / 64];
  __shared__ unsigned long long bsum3[3];
  const int64_t n = fill_n(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * FBM + (int64_t)wave * 64 * FKM;
  int32_t f[FKM];
  bool add[FKM];
  int32_t wc = -1;
#pragma unroll
  for (int k = 0; k < FKM; k++) {
    const int64_t c = c0 + k * 64 + lane;
    f[k] = 0;
    add[k] = false;
    if (c < n) {
      const int32_t t = a.top[c];
      f[k] = t > 0 ? a.fid[t] : 0;
      a.map[c] = f[k];
      add[k] = c > 0 && t != c && f[k] > 0 && (int64_t)f[k] < a.ocap && a.ofeat && a.feat;
    }
    const unsigned long long act = __ballot(add[k]);
    if (wc < 0 && act) wc = __shfl(f[k], __builtin_ctzll(act), 64);
  }
  if (lane == 0) wcand[wave] = wc;
  if (threadIdx.x < 3) bsum3[threadIdx.x] = 0;
  __syncthreads();
  int32_t cand = -1;
  for (int w = 0; w < FT / 64 && cand < 0; w++) cand = wcand[w];
  unsigned long long p0 = 0, p1 = 0, p2 = 0;  // this lane's sum for the candidate
#pragma unroll
  for (int k = 0; k < FKM; k++) {
    const int64_t c = c0 + k * 64 + lane;
    unsigned long long s0 = 0, s1 = 0, s2 = 0;
    if (add[k]) {
      const Feature& g = a.feat[c];
      s0 = (unsigned long long)g.S;
      s1 = (unsigned long long)g.Sx;
      s2 = (unsigned long long)g.Sy;
    }
    const bool mine = add[k] && f[k] == cand;
    if (mine) {
      p0 += s0;
      p1 += s1;
      p2 += s2;
    }
    const bool rest = add[k] && !mine;
    const unsigned long long act = __ballot(rest);
    if (act) {
      const int ll = __builtin_ctzll(act);
      const int32_t fl = __shfl(f[k], ll, 64);
      const bool same = rest && f[k] == fl;
      const unsigned long long t0 = fill_wave_sum(same ? s0 : 0ull);
      const unsigned long long t1 = fill_wave_sum(same ? s1 : 0ull);
      const unsigned long long t2 = fill_wave_sum(same ? s2 : 0ull);
      if (lane == ll) fill_add(&a.ofeat[fl], t0, t1, t2);
      if (rest && !same) fill_add(&a.ofeat[f[k]], s0, s1, s2);
    }
  }
  p0 = fill_wave_sum(p0);
  p1 = fill_wave_sum(p1);
  p2 = fill_wave_sum(p2);
  if (lane == 0 && cand > 0 && (p0 | p1 | p2)) {
    atomicAdd(&bsum3[0], p0);
    atomicAdd(&bsum3[1], p1);
    atomicAdd(&bsum3[2], p2);
  }
  __syncthreads();
  if (threadIdx.x == 0 && cand > 0 && (bsum3[0] | bsum3[1] | bsum3[2])) fill_add(&a.ofeat[cand], bsum3[0], bsum3[1], bsum3[2]);
}

// four pixels per thread and step, grid-stride
__global__ void __launch_bounds__(FT) k_fill_labels(Args a) {
  const int64_t n = fill_n(a);
  if (!n) return;
  const int64_t nq = a.npx / 4;
  const bool vec = ((reinterpret_cast<uintptr_t>(a.labels) | reinterpret_cast<uintptr_t>(a.olabels)) & 15) == 0;
  const int64_t stride = (int64_t)gridDim.x * FT;
  for (int64_t q = (int64_t)blockIdx.x * FT + threadIdx.x; q < nq; q += stride) {
    const int64_t i = 4 * q;
    int32_t v[4];
    if (vec) {
      const int4 l = *reinterpret_cast<const int4*>(a.labels + i);
      v[0] = l.x;
      v[1] = l.y;
      v[2] = l.z;
      v[3] = l.w;
    } else {
      for (int k = 0; k < 4; k++) v[k] = a.labels[i + k];
    }
    for (int k = 0; k < 4; k++) v[k] = (uint64_t)v[k] < (uint64_t)n ? a.map[v[k]] : -1;
    if (vec) {
      int4 o;
      o.x = v[0];
      o.y = v[1];
      o.z = v[2];
      o.w = v[3];
      *reinterpret_cast<int4*>(a.olabels + i) = o;
    } else {
      for (int k = 0; k < 4; k++) a.olabels[i + k] = v[k];
    }
  }
  // the last npx % 4 pixels
  const int64_t tail = a.npx - 4 * nq;
  if (blockIdx.x == 0 && threadIdx.x < tail) {
    const int64_t i = 4 * nq + threadIdx.x;
    const int32_t v = a.labels[i];
    a.olabels[i] = (uint64_t)v < (uint64_t)n ? a.map[v] : -1;
  }
}

}  // namespace fill
}  // namespace ccl
