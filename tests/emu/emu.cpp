// emu.cpp -- TEST HARNESS ONLY: runs the HIP kernels of ccl_pipeline.h on the
// host (see hip_mock.h) for bounds checking and parity tests on small images.
// Never part of the product: libccl.so is built from ccl.hip by hipcc.
//
// usage: ccl_emu <tile-config> <single|batch> <in.bin> <out.bin>
//   in.bin : int32 n; then per image int32 w, h; int64 pitch; uint8 [h*pitch]
//   out.bin: per image int64 n_labels, euler; int32 labels[h*w];
//            then n_labels x (int64 xmin,xmax,ymin,ymax,S,Sx,Sy; int32 parent; int32 color)
#include <stdio.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>

#include <vector>

#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#define EMU_ASAN 1
#else
#define EMU_ASAN 0
#endif

#include "../../paper_2006_09299_amd/csrc/ccl_pipeline.h"

// Fiber switch (x86-64 System V): push the callee-saved registers on the
// current stack, store its pointer in *save, load the other stack's pointer,
// pop its registers and return into it.  Unlike swapcontext it makes no
// system call (swapcontext saves and restores the signal mask on every
// switch, which was most of the harness's run time).
extern "C" void emu_switch(void** save, void* load);
asm(R"(
  .text
  .globl emu_switch
  .type emu_switch, @function
emu_switch:
  pushq %rbp
  pushq %rbx
  pushq %r12
  pushq %r13
  pushq %r14
  pushq %r15
  movq %rsp, (%rdi)
  movq %rsi, %rsp
  popq %r15
  popq %r14
  popq %r13
  popq %r12
  popq %rbx
  popq %rbp
  ret
  .size emu_switch, .-emu_switch
)");

namespace {

constexpr size_t STACK = 512 * 1024;
enum { RUNNABLE, WAITING, DONE };

struct Fiber {
  void* sp;  // saved stack pointer while switched out
  unsigned tid;
  int state;
  int wait_scope;  // 0: block, 1 + wave: wave
  char* stack;
};

struct Sched {
  void* main_sp;
  std::vector<Fiber> f;
  std::vector<char*> stacks;
  unsigned cur = 0;
  emu_dim bidx{0, 0, 0}, bdim{1, 1, 1}, gdim{1, 1, 1};
  std::function<void()> body;
  unsigned long long xchg[16][64];
  const void* main_stack_bottom = nullptr;
  size_t main_stack_size = 0;
  int sched = 0;                 // 0 thread order, 1 reverse, 2 pseudo-random
  unsigned long long rng = 1;
} S;

void* fake_main = nullptr;

void fiber_entry() {
#if EMU_ASAN
  __sanitizer_finish_switch_fiber(nullptr, &S.main_stack_bottom, &S.main_stack_size);
#endif
  S.body();
  Fiber& me = S.f[S.cur];
  me.state = DONE;
  S.xchg[me.tid / 64][me.tid % 64] = 0;
#if EMU_ASAN
  __sanitizer_start_switch_fiber(nullptr, S.main_stack_bottom, S.main_stack_size);
#endif
  emu_switch(&me.sp, S.main_sp);  // never resumed
  abort();
}

// first frame of a fiber (entered by emu_switch's return, as if called)
extern "C" void emu_fiber_start() { fiber_entry(); }

void yield_to_main() {
  Fiber& me = S.f[S.cur];
#if EMU_ASAN
  void* fake = nullptr;
  __sanitizer_start_switch_fiber(&fake, S.main_stack_bottom, S.main_stack_size);
#endif
  emu_switch(&me.sp, S.main_sp);
#if EMU_ASAN
  __sanitizer_finish_switch_fiber(fake, &S.main_stack_bottom, &S.main_stack_size);
#endif
}

void wait_on(int scope) {
  Fiber& me = S.f[S.cur];
  me.state = WAITING;
  me.wait_scope = scope;
  yield_to_main();
}

void run_block(unsigned block, unsigned nthreads) {
  if (S.stacks.size() < nthreads) {
    while (S.stacks.size() < nthreads) S.stacks.push_back(static_cast<char*>(malloc(STACK)));
  }
  S.f.assign(nthreads, Fiber());
  S.bdim = emu_dim{nthreads, 1, 1};
  S.bidx = emu_dim{block, 0, 0};
  memset(S.xchg, 0, sizeof(S.xchg));
  for (unsigned t = 0; t < nthreads; t++) {
    Fiber& fb = S.f[t];
    fb.tid = t;
    fb.state = RUNNABLE;
    fb.stack = S.stacks[t];
    // initial frame: six zero registers, then emu_fiber_start as the return
    // address, then a null return address for it (it never returns), with
    // the stack 16-byte aligned at the call
    void** p = reinterpret_cast<void**>((reinterpret_cast<uintptr_t>(fb.stack) + STACK) & ~(uintptr_t)15);
    *--p = nullptr;
    *--p = reinterpret_cast<void*>(&emu_fiber_start);
    for (int k = 0; k < 6; k++) *--p = nullptr;
    fb.sp = p;
  }
  const unsigned nwaves = (nthreads + 63) / 64;
  // order in which runnable fibers run after each barrier release: thread
  // order, reverse order, or a fresh pseudo-random permutation each pass
  // (EMU_SCHED = fwd | rev | <seed>), so that code reading shared state right
  // after a barrier meets other threads that have already gone on
  std::vector<unsigned> order(nthreads);
  for (unsigned t = 0; t < nthreads; t++) order[t] = S.sched == 1 ? nthreads - 1 - t : t;
  for (;;) {
    bool ran = false;
    if (S.sched >= 2)
      for (unsigned t = nthreads; t > 1; t--) {
        S.rng = S.rng * 6364136223846793005ull + 1442695040888963407ull;
        unsigned k = (unsigned)((S.rng >> 33) % t);
        unsigned tmp = order[t - 1];
        order[t - 1] = order[k];
        order[k] = tmp;
      }
    for (unsigned oi = 0; oi < nthreads; oi++) {
      const unsigned t = order[oi];
      if (S.f[t].state != RUNNABLE) continue;
      S.cur = t;
      ran = true;
#if EMU_ASAN
      void* fake = nullptr;
      __sanitizer_start_switch_fiber(&fake, S.f[t].stack, STACK);
#endif
      emu_switch(&S.main_sp, S.f[t].sp);
#if EMU_ASAN
      __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
    }
    bool all_done = true;
    for (auto& fb : S.f) all_done &= fb.state == DONE;
    if (all_done) return;
    if (ran) continue;
    // release a barrier whose live members all wait on it
    bool released = false;
    for (int scope = 0; scope <= (int)nwaves && !released; scope++) {
      bool any = false, all = true;
      for (auto& fb : S.f) {
        bool member = scope == 0 || (int)(fb.tid / 64) == scope - 1;
        if (!member || fb.state == DONE) continue;
        any = true;
        if (!(fb.state == WAITING && fb.wait_scope == scope)) all = false;
      }
      if (any && all) {
        for (auto& fb : S.f) {
          bool member = scope == 0 || (int)(fb.tid / 64) == scope - 1;
          if (member && fb.state == WAITING && fb.wait_scope == scope) fb.state = RUNNABLE;
        }
        released = true;
      }
    }
    if (!released) {
      fprintf(stderr, "emu: barrier deadlock in block %u\n", block);
      abort();
    }
  }
}

struct EmuLauncher {
  template <class... P, class... A>
  void launch(void (*kernel)(P...), int64_t grid, int block, A... args) {
    if (grid <= 0) return;
    S.gdim = emu_dim{(unsigned)grid, 1, 1};
    S.body = [&]() { kernel(args...); };
    for (int64_t b = 0; b < grid; b++) run_block((unsigned)b, (unsigned)block);
  }
};

}  // namespace

emu_dim emu_thread_idx() { return emu_dim{S.f[S.cur].tid, 0, 0}; }
emu_dim emu_block_idx() { return S.bidx; }
emu_dim emu_block_dim() { return S.bdim; }
emu_dim emu_grid_dim() { return S.gdim; }
void emu_block_barrier() { wait_on(0); }
int emu_block_vote_and(int pred) {
  // count the live threads voting false; two barriers keep rounds apart
  static int falses = 0;
  static int phase = 0;
  (void)phase;
  emu_block_barrier();
  if (S.f[S.cur].tid == 0) falses = 0;
  emu_block_barrier();
  if (!pred) falses++;
  emu_block_barrier();
  int r = falses == 0;
  emu_block_barrier();
  return r;
}
void emu_wave_exchange(unsigned long long v, unsigned long long* all64) {
  unsigned tid = S.f[S.cur].tid;
  unsigned wave = tid / 64;
  S.xchg[wave][tid % 64] = v;
  wait_on(1 + (int)wave);
  memcpy(all64, S.xchg[wave], sizeof(unsigned long long) * 64);
  wait_on(1 + (int)wave);
}

namespace {

struct Image {
  int32_t w, h;
  int64_t pitch;
  std::vector<uint8_t> data;
  // outputs
  std::vector<int32_t> labels;
  std::vector<ccl::Feature> feat;
  std::vector<int32_t> parent;
  std::vector<uint8_t> color;
  int64_t counts[2];
};

bool no_labels = false;  // EMU_NOLABELS=1: the features-only mode (no label image)

template <class T>
void run_images(std::vector<Image>& ims, bool batch) {
  for (auto& im : ims) {
    int64_t cap = (int64_t)im.w * im.h + 1;
    im.labels.assign((size_t)im.w * im.h, -7);
    im.feat.assign((size_t)cap, ccl::Feature{-7, -7, -7, -7, -7, -7, -7});
    im.parent.assign((size_t)cap, -7);
    im.color.assign((size_t)cap, 7);
    im.counts[0] = im.counts[1] = -7;
  }
  auto desc_of = [](Image& im) {
    ccl::ImgDesc d;
    memset(&d, 0, sizeof(d));
    d.img = im.data.data();
    d.pitch = im.pitch;
    d.w = im.w;
    d.h = im.h;
    d.labels = no_labels ? nullptr : im.labels.data();
    d.feat = im.feat.data();
    d.parent = im.parent.data();
    d.color = im.color.data();
    d.cap = (int64_t)im.w * im.h + 1;
    d.counts = im.counts;
    d.flags = 0;
    if ((reinterpret_cast<uintptr_t>(d.img) & 15) == 0 && (d.pitch & 15) == 0) d.flags |= ccl::DF_VEC_IN;
    if (d.labels && (reinterpret_cast<uintptr_t>(d.labels) & 15) == 0 && (d.w & 3) == 0) d.flags |= ccl::DF_VEC_LAB;
    return d;
  };
  EmuLauncher L;
  auto run = [&](std::vector<ccl::ImgDesc>& ds) {
    int64_t tiles = 0, nodes = 0, cells = 0, blocks = 0, items = 0, supers = 0;
    for (auto& d : ds) ccl::place_image<T>(d, tiles, nodes, cells, blocks, items, supers);
    ccl::Layout lay = ccl::make_layout<T>(tiles, nodes, cells, blocks);
    std::vector<unsigned char> ws(lay.bytes);
    memset(ws.data(), 0xA5, ws.size());  // garbage: the path must not rely on zeroed scratch
    ccl::Work wk = ccl::make_work(lay, ws.data());
    if (ds.size() == 1 && !batch) {
      ccl::OneImage src{ds[0]};
      ccl::enqueue<T, true>(L, src, wk, tiles, items, blocks, supers);
    } else {
      ccl::ManyImages src{ds.data(), (int32_t)ds.size()};
      if (tiles % 2) ccl::enqueue<T, false>(L, src, wk, tiles, items, blocks, supers);
      else ccl::enqueue<T, true>(L, src, wk, tiles, items, blocks, supers);
    }
  };
  if (batch) {
    std::vector<ccl::ImgDesc> ds;
    for (auto& im : ims) ds.push_back(desc_of(im));
    run(ds);
  } else {
    for (auto& im : ims) {
      std::vector<ccl::ImgDesc> ds{desc_of(im)};
      run(ds);
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  if (argc != 5) {
    fprintf(stderr, "usage: %s <tile-config> <single|batch> <in.bin> <out.bin>\n", argv[0]);
    return 2;
  }
  FILE* fi = fopen(argv[3], "rb");
  if (!fi) return 3;
  int32_t n = 0;
  if (fread(&n, 4, 1, fi) != 1) return 3;
  std::vector<Image> ims((size_t)n);
  for (auto& im : ims) {
    if (fread(&im.w, 4, 1, fi) != 1 || fread(&im.h, 4, 1, fi) != 1 || fread(&im.pitch, 8, 1, fi) != 1) return 3;
    // 16-byte aligned rows when the pitch allows it (the vector path), else not
    im.data.resize((size_t)im.h * im.pitch);
    if (fread(im.data.data(), 1, im.data.size(), fi) != im.data.size()) return 3;
  }
  fclose(fi);
  bool batch = strcmp(argv[2], "batch") == 0;
  if (const char* e = getenv("EMU_SCHED")) {
    if (strcmp(e, "rev") == 0) S.sched = 1;
    else if (strcmp(e, "fwd") != 0) {
      S.sched = 2;
      S.rng = strtoull(e, nullptr, 10) * 2 + 1;
    }
  }
  if (const char* e = getenv("EMU_NOLABELS")) no_labels = strcmp(e, "1") == 0;
  int cfg = atoi(argv[1]);
  switch (cfg) {
    case 0: run_images<ccl::Tile<32, 128>>(ims, batch); break;
    case 1: run_images<ccl::Tile<4, 64>>(ims, batch); break;
    case 2: run_images<ccl::Tile<3, 64>>(ims, batch); break;
    case 3: run_images<ccl::Tile<5, 192>>(ims, batch); break;
    case 4: run_images<ccl::Tile<64, 64>>(ims, batch); break;
    case 5: run_images<ccl::Tile<1, 64>>(ims, batch); break;
    case 6: run_images<ccl::Tile<16, 128, 512>>(ims, batch); break;
    case 7: run_images<ccl::Tile<64, 128>>(ims, batch); break;  // relabeling with 512 threads
    case 8: run_images<ccl::Tile<32, 128, 256, false>>(ims, batch); break;  // 4-adjacent foreground
    case 9: run_images<ccl::Tile<4, 64, 256, false>>(ims, batch); break;
    // merge schedules: 2 x 2 and 8 x 8 super-tiles, small root-reduction groups
    case 10: run_images<ccl::Tile<4, 64, 256, true, 2>>(ims, batch); break;
    case 11: run_images<ccl::Tile<4, 64, 256, true, 8, 4>>(ims, batch); break;
    case 12: run_images<ccl::Tile<3, 64, 256, true, 8, 1>>(ims, batch); break;
    // root-reduction groups of more than one wave of tiles
    case 13: run_images<ccl::Tile<4, 64, 256, true, 4, 128>>(ims, batch); break;
    case 14: run_images<ccl::Tile<3, 64, 256, true, 4, 256>>(ims, batch); break;
    default: fprintf(stderr, "bad tile config\n"); return 2;
  }
  FILE* fo = fopen(argv[4], "wb");
  if (!fo) return 4;
  for (auto& im : ims) {
    fwrite(im.counts, 8, 2, fo);
    fwrite(im.labels.data(), 4, im.labels.size(), fo);
    int64_t nl = im.counts[0];
    if (nl < 0 || nl > (int64_t)im.feat.size()) nl = 0;
    for (int64_t k = 0; k < nl; k++) {
      const ccl::Feature& f = im.feat[(size_t)k];
      int64_t v[7] = {f.xmin, f.xmax, f.ymin, f.ymax, f.S, f.Sx, f.Sy};
      fwrite(v, 8, 7, fo);
      int32_t pc[2] = {im.parent[(size_t)k], (int32_t)im.color[(size_t)k]};
      fwrite(pc, 4, 2, fo);
    }
  }
  fclose(fo);
  return 0;
}
