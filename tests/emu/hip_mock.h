// hip_mock.h -- TEST HARNESS ONLY.  Lets the HIP kernel source of
// paper_2006_09299_amd/csrc/ccl_pipeline.h compile and run on the host
// (g++ with AddressSanitizer / UBSan) so that every memory access of every
// kernel is bounds-checked and the results compared with the oracle before a
// GPU runs them.  Threads of a workgroup are cooperative fibers (ucontext);
// a workgroup barrier switches fibers; wave operations (shuffle, ballot)
// synchronise the 64 fibers of a wave.  Atomics are plain read-modify-writes
// (fibers never preempt each other).  Blocks of a grid run one after another.
#pragma once

#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <functional>

#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __launch_bounds__(...)

#define __HIP_MEMORY_SCOPE_WORKGROUP 3
#define __HIP_MEMORY_SCOPE_AGENT 4

struct uint4 {
  unsigned x, y, z, w;
};
struct int4 {
  int x, y, z, w;
};
struct emu_dim {
  unsigned x, y, z;
};

emu_dim emu_thread_idx();
emu_dim emu_block_idx();
emu_dim emu_block_dim();
emu_dim emu_grid_dim();
void emu_block_barrier();
void emu_wave_exchange(unsigned long long v, unsigned long long* all64);

#define threadIdx (emu_thread_idx())
#define blockIdx (emu_block_idx())
#define blockDim (emu_block_dim())
#define gridDim (emu_grid_dim())

// fibers of a wave meet at wave operations; a fence has no host meaning
#define __builtin_amdgcn_fence(...) ((void)0)

inline void __syncthreads() { emu_block_barrier(); }
int emu_block_vote_and(int pred);
inline int __syncthreads_and(int pred) { return emu_block_vote_and(pred); }

template <class V>
inline V __shfl_up(V v, unsigned d, int = 64) {
  unsigned long long all[64], mine = 0;
  memcpy(&mine, &v, sizeof(V));
  emu_wave_exchange(mine, all);
  unsigned lane = emu_thread_idx().x % 64;
  if (lane < d) return v;
  V r;
  memcpy(&r, &all[lane - d], sizeof(V));
  return r;
}
template <class V>
inline V __shfl(V v, int src, int = 64) {
  unsigned long long all[64], mine = 0;
  memcpy(&mine, &v, sizeof(V));
  emu_wave_exchange(mine, all);
  V r;
  memcpy(&r, &all[src & 63], sizeof(V));
  return r;
}
inline unsigned long long __ballot(int pred) {
  unsigned long long all[64];
  emu_wave_exchange(pred ? 1ull : 0ull, all);
  unsigned long long m = 0;
  for (unsigned k = 0; k < 64; k++)
    if (all[k] == 1ull) m |= 1ull << k;
  return m;
}

// clang knows the __hip_atomic_* names as builtins even for the host
#define __hip_atomic_load emu_atomic_load
#define __hip_atomic_store emu_atomic_store
#define __hip_atomic_fetch_min emu_atomic_fetch_min
#define __hip_atomic_compare_exchange_strong emu_atomic_cas

template <class P>
inline P emu_atomic_load(const P* p, int, int) {
  return *p;
}
template <class P, class V>
inline void emu_atomic_store(P* p, V v, int, int) {
  *p = (P)v;
}
template <class P, class V>
inline P emu_atomic_fetch_min(P* p, V v, int, int) {
  P old = *p;
  if ((P)v < old) *p = (P)v;
  return old;
}

template <class P, class V>
inline bool emu_atomic_cas(P* p, P* expected, V desired, int, int, int) {
  if (*p == *expected) {
    *p = (P)desired;
    return true;
  }
  *expected = *p;
  return false;
}

template <class P, class V>
inline P atomicMin(P* p, V v) {
  P old = *p;
  if ((P)v < old) *p = (P)v;
  return old;
}
template <class P, class V>
inline P atomicMax(P* p, V v) {
  P old = *p;
  if ((P)v > old) *p = (P)v;
  return old;
}
template <class P, class V>
inline P atomicAdd(P* p, V v) {
  P old = *p;
  *p = (P)(old + (P)v);
  return old;
}
template <class P, class V, class W>
inline P atomicCAS(P* p, V cmp, W v) {
  P old = *p;
  if (old == (P)cmp) *p = (P)v;
  return old;
}
template <class P, class V>
inline P atomicOr(P* p, V v) {
  P old = *p;
  *p = (P)(old | (P)v);
  return old;
}
